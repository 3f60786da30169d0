"""Simple-update imaginary-time evolution of the vectorised PEPS (test
infrastructure: the plain reference for the device's simple update).

The paper's alternative for the highest temperatures (the paragraph on the
simple-update method, after Appendix A): near beta = 0 the state is close to
the product state |I>, environments matter little, and the simple update of
Jiang, Weng and Xiang evolves the PEPS by Trotter gates with bond weights
lambda standing in for the environment, before SR takes over.

One step of tau approximates exp(-tau calH) (the same time step as one SR
step, so n steps reach beta_phys = 4 n tau): first-order Trotter over the
nearest-neighbour bonds in four groups, horizontal bonds with c even, c odd,
vertical bonds with r even, r odd, each group in row-major order of its
bonds.  The gate of a bond with coupling J is exp(-tau calH_b) =
exp(-tau J h) (x) exp(-tau J h^T) on the doubled digits S = s d + s' of its
two sites (h = S_i.S_j; ket digits by the first factor, bra digits by the
second).  Update of a bond (i, j):
  1. multiply every other leg of T_i and T_j by its bond weight;
  2. Theta = sum_b T_i[.., b] lambda_b T_j[.., b] with the gate applied on
     (S_i, S_j);
  3. SVD of Theta as (legs of i, S_i) x (S_j, legs of j), keep the D largest
     values (no threshold; zero padding if the rank is smaller);
  4. lambda_b <- kept values / their maximum; T_i <- U, T_j <- V^T;
  5. divide the other legs by their weights again, a weight below
     LAMBDA_CUT times the largest weight of its bond counting as zero (its
     inverse is 0).
`absorb` returns the plain PEPS with sqrt(lambda_b) on both ends of every
bond, the input of sampling and SR.

Bond weights are stored [n_bonds][D]: horizontal bonds row-major, then
vertical bonds row-major.  Spin models with J2 = 0 only (no gates on
next-nearest-neighbour bonds).
"""
from __future__ import annotations

import numpy as np

from .lattice import MODEL_HEISENBERG

LAMBDA_CUT = 1e-12

# leg positions in T[S][l][u][r][d]
_L, _U, _R, _Dn = 1, 2, 3, 4


def bonds(lat):
    """[(i, j, leg of i, leg of j, bond index)] in the update order."""
    hs = [((r, c), (r, c + 1)) for r in range(lat.L1) for c in range(lat.L2 - 1)]
    vs = [((r, c), (r + 1, c)) for r in range(lat.L1 - 1) for c in range(lat.L2)]
    index = {b: k for k, b in enumerate(hs + vs)}
    order = []
    for par in (0, 1):
        order += [(a, b, _R, _L) for (a, b) in hs if a[1] % 2 == par]
    for par in (0, 1):
        order += [(a, b, _Dn, _U) for (a, b) in vs if a[0] % 2 == par]
    return [(lat.site(*a), lat.site(*b), la, lb, index[(a, b)]) for (a, b, la, lb) in order]


def n_bonds(lat):
    return lat.L1 * (lat.L2 - 1) + (lat.L1 - 1) * lat.L2


def _leg_bonds(lat):
    """leg_bond[i][leg] = bond index on that leg of site i, or -1."""
    out = [[-1] * 5 for _ in range(lat.N)]
    for (i, j, li, lj, k) in bonds(lat):
        out[i][li] = k
        out[j][lj] = k
    return out


def gate(lat, tau, J):
    """exp(-tau calH_b) as a (d^2 d^2) x (d^2 d^2) matrix on (S_i, S_j)."""
    if lat.model != MODEL_HEISENBERG or lat.d != 2:
        raise ValueError("simple update: spin-1/2 Heisenberg only")
    sz = np.array([[0.5, 0.0], [0.0, -0.5]])
    sp = np.array([[0.0, 1.0], [0.0, 0.0]])
    h = J * (np.kron(sz, sz) + 0.5 * (np.kron(sp, sp.T) + np.kron(sp.T, sp)))   # on (s_i, s_j)
    w, v = np.linalg.eigh(h)
    e = (v * np.exp(-tau * w)) @ v.T                                          # exp(-tau h)
    et = e.T                                                                  # exp(-tau h^T)
    d = 2
    G = np.zeros((16, 16))
    for si in range(d):
        for spi in range(d):
            for sj in range(d):
                for spj in range(d):
                    for ti in range(d):
                        for tpi in range(d):
                            for tj in range(d):
                                for tpj in range(d):
                                    G[(si * d + spi) * 4 + (sj * d + spj), (ti * d + tpi) * 4 + (tj * d + tpj)] = \
                                        e[si * d + sj, ti * d + tj] * et[spi * d + spj, tpi * d + tpj]
    return G


def _site(lat, theta, i):
    return lat.site_tensor(theta, i // lat.L2, i % lat.L2)


def _weights(lat, lam, i, legbond, skip, inverse):
    """Per-leg weight vectors of site i (ones on boundary legs and on `skip`)."""
    T_dims = lat.leg_dims(i // lat.L2, i % lat.L2)
    ws = []
    for leg in (_L, _U, _R, _Dn):
        k = legbond[i][leg]
        n = T_dims[leg - 1]
        if k < 0 or leg == skip:
            ws.append(np.ones(n))
            continue
        v = lam[k][:n]
        if inverse:
            cut = LAMBDA_CUT * np.max(v)
            v = np.where(v > cut, 1.0 / np.where(v > cut, v, 1.0), 0.0)
        ws.append(v)
    return ws


def _scale(T, ws):
    return T * ws[0][None, :, None, None, None] * ws[1][None, None, :, None, None] * \
        ws[2][None, None, None, :, None] * ws[3][None, None, None, None, :]


def update_bond(lat, theta, lam, i, j, li, lj, k, G, legbond):
    Ti = _site(lat, theta, i)
    Tj = _site(lat, theta, j)
    D = Ti.shape[li]
    Ai = _scale(Ti, _weights(lat, lam, i, legbond, li, False))
    Aj = _scale(Tj, _weights(lat, lam, j, legbond, lj, False))
    # move the bond leg last (i) / first after S (j)
    Ai = np.moveaxis(Ai, li, -1)                  # [S_i, other..., b]
    Aj = np.moveaxis(Aj, lj, 1)                   # [S_j, b, other...]
    oi, oj = Ai.shape[1:-1], Aj.shape[2:]
    Mi = np.moveaxis(Ai, 0, -2).reshape(-1, 4, D)  # [(other_i), S_i, b]
    Mj = Aj.reshape(4, D, -1)                      # [S_j, b, (other_j)]
    theta2 = np.einsum("xsb,b,tby->xsty", Mi, lam[k], Mj)
    theta2 = np.einsum("uvst,xsty->xuvy", G.reshape(4, 4, 4, 4), theta2)
    ni, nj = theta2.shape[0], theta2.shape[3]
    U, s, Vt = np.linalg.svd(theta2.reshape(ni * 4, 4 * nj), full_matrices=False)
    keep = min(D, s.size)
    lam_new = np.zeros(D)
    lam_new[:keep] = s[:keep] / s[0] if s[0] > 0 else 0.0
    Un = np.zeros((ni * 4, D))
    Vn = np.zeros((D, 4 * nj))
    Un[:, :keep] = U[:, :keep]
    Vn[:keep] = Vt[:keep]
    Ti_new = np.moveaxis(Un.reshape(oi + (4, D)), -2, 0)    # [S_i, other..., b]
    Ti_new = np.moveaxis(Ti_new, -1, li)
    Tj_new = np.moveaxis(Vn.reshape((D, 4) + oj), 1, 0)     # [S_j, b, other...]
    Tj_new = np.moveaxis(Tj_new, 1, lj)
    lam[k] = lam_new
    Ti_new = _scale(Ti_new, _weights(lat, lam, i, legbond, li, True))
    Tj_new = _scale(Tj_new, _weights(lat, lam, j, legbond, lj, True))
    Ti[...] = Ti_new
    Tj[...] = Tj_new


def su_step(lat, theta, lam, tau):
    """One simple-update step of tau in place on theta (packed) and lam."""
    if lat.J2 != 0.0:
        raise ValueError("simple update: nearest-neighbour bonds only (J2 = 0)")
    G = gate(lat, tau, lat.J1)
    legbond = _leg_bonds(lat)
    for (i, j, li, lj, k) in bonds(lat):
        update_bond(lat, theta, lam, i, j, li, lj, k, G, legbond)


def absorb(lat, theta, lam):
    """Plain PEPS: sqrt(lambda) on both ends of every bond."""
    out = np.array(theta, dtype=np.float64, copy=True)
    legbond = _leg_bonds(lat)
    sq = np.sqrt(np.asarray(lam))
    for i in range(lat.N):
        T = _site(lat, out, i)
        T[...] = _scale(T, _weights(lat, sq, i, legbond, -1, False))
    return out
