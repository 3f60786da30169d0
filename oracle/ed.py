"""Exact diagonalisation and thermal energies (reference values for the
cooling loop; the Benchmark section compares with ED on a 4x4 J1-J2 lattice).

Heisenberg: H is block diagonal in the number of up spins; each block is
built from bit strings (bit i = 1 means spin i is down, site 0 = most
significant bit, matching the dense builder) and diagonalised with
numpy.linalg.eigh.  Thermal energy at inverse temperature beta:
    E(beta) = sum_n E_n exp(-beta (E_n - E_0)) / sum_n exp(-beta (E_n - E_0)).
"""
from __future__ import annotations

from itertools import combinations

import numpy as np


def spin_pairs(lat):
    pairs = [(lat.site(*a), lat.site(*b), lat.J1) for a, b in lat.bonds_h() + lat.bonds_v()]
    if lat.J2 != 0.0:
        pairs += [(lat.site(*a), lat.site(*b), lat.J2) for a, b in lat.bonds_d()]
    return pairs


def spin_sector_matrix(lat, n_down):
    N = lat.N
    states = []
    for downs in combinations(range(N), n_down):
        x = 0
        for i in downs:
            x |= 1 << (N - 1 - i)
        states.append(x)
    states.sort()
    index = {x: k for k, x in enumerate(states)}
    H = np.zeros((len(states), len(states)))
    pairs = spin_pairs(lat)
    for k, x in enumerate(states):
        for i, j, J in pairs:
            bi = (x >> (N - 1 - i)) & 1
            bj = (x >> (N - 1 - j)) & 1
            H[k, k] += J * (0.25 if bi == bj else -0.25)
            if bi != bj:
                y = x ^ (1 << (N - 1 - i)) ^ (1 << (N - 1 - j))
                H[index[y], k] += 0.5 * J
    return H


def spin_spectrum(lat):
    """All eigenvalues of the J1-J2 Hamiltonian, sector by sector."""
    ev = []
    for nd in range(lat.N + 1):
        ev.append(np.linalg.eigvalsh(spin_sector_matrix(lat, nd)))
    return np.concatenate(ev)


def spin_spectrum_sectors(lat):
    """[(n_down, eigenvalues)] of the J1-J2 Hamiltonian; M_z = (N - 2 n_down) / 2
    is constant on each sector."""
    return [(nd, np.linalg.eigvalsh(spin_sector_matrix(lat, nd))) for nd in range(lat.N + 1)]


def thermal_mz2(sectors, N, beta):
    """Canonical <M_z^2> at inverse temperature beta (array-valued): M_z is
    conserved, so each eigenstate of sector n_down contributes
    ((N - 2 n_down) / 2)^2."""
    e0 = min(float(ev.min()) for _, ev in sectors)
    beta = np.atleast_1d(np.asarray(beta, dtype=np.float64))
    out = np.empty_like(beta)
    for k, b in enumerate(beta):
        num = 0.0
        den = 0.0
        for nd, ev in sectors:
            w = np.exp(-b * (ev - e0)).sum()
            num += w * ((N - 2 * nd) / 2.0) ** 2
            den += w
        out[k] = num / den
    return out


def thermal_energy(evals, beta):
    """Canonical internal energy at inverse temperature beta (array-valued)."""
    evals = np.asarray(evals, dtype=np.float64)
    e0 = evals.min()
    beta = np.atleast_1d(np.asarray(beta, dtype=np.float64))
    out = np.empty_like(beta)
    for k, b in enumerate(beta):
        w = np.exp(-b * (evals - e0))
        out[k] = float(np.dot(w, evals) / w.sum())
    return out


def thermal_specific_heat(evals, beta, N):
    """Specific heat per site C_v = beta^2 (<E^2> - <E>^2) / N, the canonical
    fluctuation formula (equal to -beta^2 dE/dbeta / N)."""
    evals = np.asarray(evals, dtype=np.float64)
    e0 = evals.min()
    beta = np.atleast_1d(np.asarray(beta, dtype=np.float64))
    out = np.empty_like(beta)
    for k, b in enumerate(beta):
        w = np.exp(-b * (evals - e0))
        w /= w.sum()
        m = float(np.dot(w, evals))
        out[k] = b * b * float(np.dot(w, (evals - m) ** 2)) / N
    return out
