"""Thermal observables on the device (local values of M_z, M_z^2, particle
number and double occupancy) against the oracle: every value is a multiple
of 1/8, so the comparison is bit-exact.  The whole-loop physics check of
<M_z^2> against exact diagonalisation is in tests/test_gpu_cooling.py."""
import sys

import numpy as np
import pytest

import synth
from oracle import observables
from oracle.lattice import MODEL_HUBBARD, Lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


@pytest.mark.parametrize("model", ["spin", "hubbard"])
def test_observables_bit_exact(model):
    dev = _dev()
    import paper_2409_05285_amd as p
    print("[case] observables", model, flush=True)
    sys.stdout.flush()
    if model == "spin":
        lat = Lattice(5, 7, D=2, chi=4)
        desc = p.Desc(5, 7, 2, 4)
        cfg = np.concatenate([synth.configs_uniform(300, lat.N, 2, seed=71), synth.configs_diagonal(3, lat.N, 2, seed=72)])
    else:
        lat = Lattice(4, 6, D=2, chi=4, d=4, model=MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0)
        desc = p.Desc(4, 6, 2, 4, d=4, model=p.MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0)
        cfg = synth.configs_uniform(300, lat.N, 4, seed=73)
    got = p.peps_observables_batch(desc, torch.tensor(cfg, device=dev)).cpu().numpy()
    ref = observables.local_values_batch(lat, cfg)
    assert np.array_equal(got, ref)
    # empty batch: a no-op
    assert p.peps_observables_batch(desc, torch.zeros((0, lat.N), dtype=torch.uint8, device=dev)).shape == (0, 4)
