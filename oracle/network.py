"""Exact (untruncated) contraction of the single-layer network rho_theta(S).

Method section, Eq. (4): rho_theta(S) is the full contraction of the site
matrices T_i^{S_i}.  Here it is evaluated with a dense row-transfer tensor
over the down legs of the rows absorbed so far (dimension D^{L2}), absorbed
one site at a time.  No QR or SVD is involved, so this is the definition
written out; it is only feasible for small lattices (D^{L2} up to a few
thousand).
"""
from __future__ import annotations

import itertools

import numpy as np


def amplitude(lat, theta, config):
    """rho_theta(S) for one configuration, exact."""
    cfg = np.asarray(config).reshape(lat.L1, lat.L2)
    V = np.ones((1,) * lat.L2)          # up legs of row 0 all have dimension 1
    for r in range(lat.L1):
        W = lat.row_slices(theta, cfg, r)
        X = V.reshape((1, 1) + V.shape)  # [done (empty), l0, u0, u1, ...]
        done = 1
        for c in range(lat.L2):
            rest = int(np.prod(X.shape[3:])) if X.ndim > 3 else 1
            Xc = X.reshape(done, X.shape[1], X.shape[2], rest)
            # contract the incoming horizontal leg l and the up leg u of site c
            Y = np.einsum("aluB,lurd->adrB", Xc, W[c])
            done *= Y.shape[1]
            tail = X.shape[3:]
            X = Y.reshape((done, Y.shape[2]) + tuple(tail))
        # the right leg of the last site has dimension 1
        V = X.reshape(tuple(W[c].shape[3] for c in range(lat.L2)))
    return float(V.reshape(()))


def all_configs(lat):
    """Every configuration S in [0, d^2)^N, as an array [d2^N, N]."""
    return np.array(list(itertools.product(range(lat.d2), repeat=lat.N)), dtype=np.int64)


def density_matrix(lat, theta):
    """The operator rho with entries rho[s, s'] = rho_theta(S), where
    s = (s_1..s_N) and s' = (s'_1..s'_N) are read as base-d numbers with site 1
    most significant (Method section, Eq. (2): vectorisation |s>|s'>)."""
    d, N = lat.d, lat.N
    rho = np.zeros((d ** N, d ** N))
    for S in all_configs(lat):
        s = 0
        sp = 0
        for Si in S:
            s = s * d + lat.ket(Si)
            sp = sp * d + lat.bra(Si)
        rho[s, sp] = amplitude(lat, theta, S)
    return rho
