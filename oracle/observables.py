"""Thermal observables from the same samples (test infrastructure: the
plain reference for the device's observable kernel).

The Benchmark section reports, besides the internal energy, the uniform
magnetic susceptibility chi = beta <M_z^2> / N with <M_z>^2 set to zero
(Heisenberg), and the double occupancy D = sum_i <n_i,up n_i,dn> / N
(Hubbard).  In the vectorised form the thermal expectation of an operator A
is Tr(rho rho^T A) / Tr(rho rho^T) (rho rho^T proportional to exp(-beta H));
for A diagonal in the computational basis both Tr(rho rho^T A) and
Tr(rho^T rho A) are sums of |rho(S)|^2 A over the ket or the bra digits, so
the local value of a diagonal A is (A(s) + A(s')) / 2 and its mean under
|rho|^2 is the symmetrised expectation (the same symmetrisation as
E_loc / 2 for the energy).

Per sample, in this order (OBS_NAMES):
  mz    (M_z(s) + M_z(s')) / 2,        M_z = sum_i S^z_i
  mz2   (M_z(s)^2 + M_z(s')^2) / 2
  n     (N(s) + N(s')) / 2,            particle number (Hubbard; 0 for spins)
  docc  (D(s) + D(s')) / 2,            D = sum_i n_i,up n_i,dn (Hubbard; 0 for spins)
Spin digit s: 0 = up (S^z = +1/2), 1 = down.  Hubbard digit s = n_up + 2 n_dn,
S^z = (n_up - n_dn) / 2.
"""
from __future__ import annotations

import numpy as np

from .lattice import MODEL_HEISENBERG, MODEL_HUBBARD

OBS_NAMES = ("mz", "mz2", "n", "docc")


def _one_side(lat, digits):
    if lat.model == MODEL_HEISENBERG:
        mz = sum(0.5 - s for s in digits)
        return mz, mz * mz, 0.0, 0.0
    if lat.model == MODEL_HUBBARD:
        mz = 0.0
        n = 0.0
        docc = 0.0
        for s in digits:
            nu, nd = s & 1, (s >> 1) & 1
            mz += 0.5 * (nu - nd)
            n += nu + nd
            docc += nu * nd
        return mz, mz * mz, n, docc
    raise ValueError("unknown model")


def local_values(lat, S):
    """The four local values of one configuration S (merged digits)."""
    S = np.asarray(S).reshape(lat.N)
    ket = _one_side(lat, [lat.ket(x) for x in S])
    bra = _one_side(lat, [lat.bra(x) for x in S])
    return np.array([(a + b) / 2.0 for a, b in zip(ket, bra)])


def local_values_batch(lat, configs):
    return np.stack([local_values(lat, S) for S in configs])


def estimate(values, weights=None):
    """Mean of each column (weighted when weights are given, Eq. A1)."""
    v = np.asarray(values, dtype=np.float64)
    if weights is None:
        return v.mean(axis=0)
    w = np.asarray(weights, dtype=np.float64)
    return (w[:, None] * v).sum(axis=0) / w.sum()


def susceptibility(mz2_mean, beta, N):
    """chi = beta <M_z^2> / N with <M_z>^2 := 0 (Benchmark section)."""
    return beta * mz2_mean / N
