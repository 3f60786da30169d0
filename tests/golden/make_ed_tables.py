"""Write the exact-diagonalisation energy tables used by the cooling checks.

Calls only the oracle (sector-by-sector ED of the 4x4 open-boundary J1-J2
model, the lattice of the Benchmark section's ED comparison) and stores
E(beta)/N and <M_z^2>(beta)/N on a grid of inverse temperatures together
with the ground-state energy.  Run:  python tests/golden/make_ed_tables.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ed  # noqa: E402
from oracle.lattice import Lattice  # noqa: E402


def table(J2):
    lat = Lattice(4, 4, D=1, chi=1, J1=1.0, J2=J2)
    sectors = ed.spin_spectrum_sectors(lat)
    ev = np.concatenate([x for _, x in sectors])
    betas = np.round(np.arange(0.0, 10.0 + 1e-9, 0.01), 10)
    e = ed.thermal_energy(ev, betas) / lat.N
    mz2 = ed.thermal_mz2(sectors, lat.N, betas) / lat.N
    return {"L1": 4, "L2": 4, "J1": 1.0, "J2": J2, "boundary": "open",
            "E0_per_site": float(ev.min() / lat.N), "dim": int(ev.size),
            "trace_H": float(ev.sum()), "trace_H2_over_dim": float((ev ** 2).mean()),
            "beta": betas.tolist(), "E_per_site": e.tolist(), "Mz2_per_site": mz2.tolist()}


if __name__ == "__main__":
    for J2, name in ((0.0, "ed_heisenberg_4x4.json"), (0.5, "ed_j1j2_4x4_j2_0.5.json")):
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(table(J2), f)
        print("wrote", name)
