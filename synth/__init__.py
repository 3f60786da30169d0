"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only produces inputs: parameter vectors and configurations.  It
holds none of the method's arithmetic (no contraction, no estimator, no
update), so it can feed both sides without coupling them.

Parameter layout (a convention, not arithmetic): sites in row-major order,
each site a block T[S][l][u][r][d] with S in [0, d^2) and a virtual leg of
dimension 1 where it points out of the open lattice, D otherwise.
"""
from __future__ import annotations

import numpy as np


def _leg_dims(L1, L2, D, r, c):
    return (1 if c == 0 else D, 1 if r == 0 else D,
            1 if c == L2 - 1 else D, 1 if r == L1 - 1 else D)


def site_shapes(L1, L2, D, d):
    return [(d * d,) + _leg_dims(L1, L2, D, r, c) for r in range(L1) for c in range(L2)]


def theta_identity(L1, L2, D, d, noise=0.0, seed=0):
    """The beta = 0 state |I> (entry [S=(s,s)][0,0,0,0] = 1 at every site)
    plus, if noise > 0, N(0, noise^2) on every element."""
    rng = np.random.Generator(np.random.Philox(seed))
    blocks = []
    for shp in site_shapes(L1, L2, D, d):
        T = np.zeros(shp)
        for s in range(d):
            T[s * d + s, 0, 0, 0, 0] = 1.0
        if noise > 0.0:
            T = T + noise * rng.standard_normal(shp)
        blocks.append(T.reshape(-1))
    return np.concatenate(blocks)


def theta_random_unit(L1, L2, D, d, seed=0):
    """i.i.d. N(0,1) entries, each site tensor scaled to unit Frobenius norm."""
    rng = np.random.Generator(np.random.Philox(seed))
    blocks = []
    for shp in site_shapes(L1, L2, D, d):
        T = rng.standard_normal(shp)
        blocks.append((T / np.linalg.norm(T)).reshape(-1))
    return np.concatenate(blocks)


def _popcount(x):
    return bin(int(x)).count("1")


def theta_random_parity_even(L1, L2, D, d, seed=0):
    """Z2-graded random tensors (the fermionic ansatz's block structure):
    a virtual index k of a leg of dimension D has parity 0 for k < D // 2
    and 1 otherwise (a leg of dimension 1 is even); the physical index
    S = s d + s' has the parity of the occupation numbers of s and s' (bit
    counts of the Hubbard digits; for d = 2 the bit of each digit).  Entries
    whose total parity is odd are zero; the rest are i.i.d. N(0,1), each
    site scaled to unit Frobenius norm."""
    rng = np.random.Generator(np.random.Philox(seed))
    blocks = []
    for shp in site_shapes(L1, L2, D, d):
        T = rng.standard_normal(shp)
        ps = np.array([(_popcount(S // d) + _popcount(S % d)) & 1 for S in range(d * d)])
        legs = [np.array([0 if (n == 1 or k < n // 2) else 1 for k in range(n)]) for n in shp[1:]]
        par = (ps[:, None, None, None, None] + legs[0][None, :, None, None, None] + legs[1][None, None, :, None, None]
               + legs[2][None, None, None, :, None] + legs[3][None, None, None, None, :]) & 1
        T = np.where(par == 0, T, 0.0)
        blocks.append((T / np.linalg.norm(T)).reshape(-1))
    return np.concatenate(blocks)


def configs_diagonal(n, N, d, seed=0):
    """n configurations with s_i = s'_i, s_i uniform (an exact sample of |I>)."""
    rng = np.random.Generator(np.random.Philox(seed))
    s = rng.integers(0, d, size=(n, N))
    return (s * d + s).astype(np.uint8)


def configs_sector(n, N, d, seed=0):
    """n configurations whose bra digits are a random permutation of the ket
    digits (equal magnetisation / particle numbers of s and s')."""
    rng = np.random.Generator(np.random.Philox(seed))
    out = np.empty((n, N), dtype=np.uint8)
    for k in range(n):
        s = rng.integers(0, d, size=N)
        sp = s[rng.permutation(N)]
        out[k] = (s * d + sp).astype(np.uint8)
    return out


def configs_uniform(n, N, d, seed=0):
    rng = np.random.Generator(np.random.Philox(seed))
    return rng.integers(0, d * d, size=(n, N)).astype(np.uint8)
