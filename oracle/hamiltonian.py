"""Local energy of the doubled generator and dense model operators.

Method section, Eq. (3): the vectorised state evolves under
    calH = H (x) I + I (x) H^T,
so <s,s'| calH |t,t'> = H_{st} delta_{s't'} + delta_{st} H_{t's'}.  Both models
used here have a real symmetric H in the chosen basis, so H^T = H and the bra
half has the same form as the ket half.

Local energy (Method section, Eq. (9)):
    E_loc(S) = sum_{S'} calH_{S S'} rho(S') / rho(S)
             = diag(S) + sum_k coeff_k * rho(S'_k) / rho(S).
`terms(lat, S)` lists the diagonal value and every off-diagonal (S'_k,
coeff_k, bond_k); the caller supplies the amplitude ratios.

Models:
  * J1-J2 Heisenberg (Benchmark section, Eq. (j1j2eq)), spin-1/2, digit
    s = 0 for up (S^z = +1/2), s = 1 for down; z = 1 - 2s;
    S_i.S_j = z_i z_j / 4 + (1/2)(flip of an anti-aligned pair).
  * Fermi-Hubbard (Benchmark section, Eq. (hubbard_model)), digit
    s = n_up + 2 n_dn; Jordan-Wigner mode order: sites row-major, up before
    down (mode 2 i + sigma).  <t| c^dag_a c_b |s> = (-1)^(number of occupied
    modes strictly between a and b).
  * Optional next-nearest-neighbour spin exchange on the Hubbard lattice,
    J2 sum_<<ij>> S_i.S_j with S^z = (n_up - n_dn)/2 and S^+_i =
    c^dag_{i,up} c_{i,dn}.  J2 = 0 is the plain Hubbard model; with t = U =
    mu = 0 and J2 = 1 the local energy is the estimator of sum_<<ij>> S_i.S_j,
    the next-nearest-neighbour spin correlation the Benchmark section reports
    for the Hubbard model (F, divided by the number of pairs).  S^+_i S^-_j is
    a product of two on-site bilinears whose modes are adjacent, so it carries
    no Jordan-Wigner sign: it swaps a singly occupied up digit with a singly
    occupied down digit.
"""
from __future__ import annotations

from functools import reduce

import numpy as np

from .lattice import MODEL_HEISENBERG, MODEL_HUBBARD


def _digits(lat, S):
    S = np.asarray(S).reshape(lat.N)
    return [lat.ket(x) for x in S], [lat.bra(x) for x in S]


def _with_digit(lat, S, changes, side):
    """Copy of S with the ket (side 0) or bra (side 1) digit of sites changed."""
    S2 = np.array(S, dtype=np.int64).reshape(lat.N).copy()
    for i, v in changes:
        s, sp = lat.ket(S2[i]), lat.bra(S2[i])
        if side == 0:
            s = v
        else:
            sp = v
        S2[i] = lat.merge(s, sp)
    return S2


def spin_bonds(lat):
    """[(i, j, J_b, kind)], kind 'h' / 'v' / 'd' (J2 bonds only when J2 != 0)."""
    out = []
    for (a, b) in lat.bonds_h():
        out.append((lat.site(*a), lat.site(*b), lat.J1, "h"))
    for (a, b) in lat.bonds_v():
        out.append((lat.site(*a), lat.site(*b), lat.J1, "v"))
    if lat.J2 != 0.0:
        for (a, b) in lat.bonds_d():
            out.append((lat.site(*a), lat.site(*b), lat.J2, "d"))
    return out


def hubbard_pairs(lat):
    out = []
    for (a, b) in lat.bonds_h():
        out.append((lat.site(*a), lat.site(*b), "h"))
    for (a, b) in lat.bonds_v():
        out.append((lat.site(*a), lat.site(*b), "v"))
    return out


def terms(lat, S):
    """(diagonal value, [(S', coeff, (i, j, kind, side))]) of calH at row S."""
    ks, bs = _digits(lat, S)
    if lat.model == MODEL_HEISENBERG:
        diag = 0.0
        off = []
        for i, j, J, kind in spin_bonds(lat):
            for side, dg in ((0, ks), (1, bs)):
                zi, zj = 1 - 2 * dg[i], 1 - 2 * dg[j]
                diag += J * 0.25 * zi * zj
                if dg[i] != dg[j]:
                    S2 = _with_digit(lat, S, [(i, dg[j]), (j, dg[i])], side)
                    off.append((S2, 0.5 * J, (i, j, kind, side)))
        return diag, off
    if lat.model == MODEL_HUBBARD:
        diag = 0.0
        for dg in (ks, bs):
            for x in dg:
                nu, nd = x & 1, (x >> 1) & 1
                diag += lat.U * nu * nd - lat.mu * (nu + nd)
        off = []
        for i, j, kind in hubbard_pairs(lat):
            for side, dg in ((0, ks), (1, bs)):
                for sg in (0, 1):
                    ni, nj = (dg[i] >> sg) & 1, (dg[j] >> sg) & 1
                    if ni == nj:
                        continue
                    # move the sigma particle between i and j; the sign counts
                    # occupied modes strictly between modes 2i+sg and 2j+sg
                    ma, mb = 2 * i + sg, 2 * j + sg
                    lo, hi = min(ma, mb), max(ma, mb)
                    between = 0
                    for m in range(lo + 1, hi):
                        between += (dg[m // 2] >> (m % 2)) & 1
                    sign = -1.0 if between % 2 else 1.0
                    newi = dg[i] ^ (1 << sg)
                    newj = dg[j] ^ (1 << sg)
                    S2 = _with_digit(lat, S, [(i, newi), (j, newj)], side)
                    off.append((S2, -lat.t * sign, (i, j, kind, side)))
        if lat.J2 != 0.0:
            for (a, b) in lat.bonds_d():
                i, j = lat.site(*a), lat.site(*b)
                for side, dg in ((0, ks), (1, bs)):
                    szi = 0.5 * ((dg[i] & 1) - ((dg[i] >> 1) & 1))
                    szj = 0.5 * ((dg[j] & 1) - ((dg[j] >> 1) & 1))
                    diag += lat.J2 * szi * szj
                    # singly occupied (digit 1 = up, 2 = down) with opposite spins
                    if dg[i] in (1, 2) and dg[j] in (1, 2) and dg[i] != dg[j]:
                        S2 = _with_digit(lat, S, [(i, dg[j]), (j, dg[i])], side)
                        off.append((S2, 0.5 * lat.J2, (i, j, "d", side)))
        return diag, off
    raise ValueError("unknown model")


def local_energy(lat, S, ratio):
    """E_loc(S) with `ratio(S2, term_info) = rho(S2) / rho(S)`."""
    diag, off = terms(lat, S)
    e = diag
    for S2, coeff, info in off:
        e += coeff * ratio(S2, info)
    return e


# ---------------------------------------------------------------------------
# Dense operators, built independently of `terms` (Kronecker products with
# explicit Jordan-Wigner strings), for identity checks on tiny lattices.

_SZ = np.array([[0.5, 0.0], [0.0, -0.5]])
_SP = np.array([[0.0, 1.0], [0.0, 0.0]])   # |up><down|, basis (up, down)
_SM = _SP.T
_I2 = np.eye(2)


def _site_op(ops, N):
    return reduce(np.kron, ops) if N else np.ones((1, 1))


def _embed(op_by_site, N, dim, ident):
    mats = [op_by_site.get(k, ident) for k in range(N)]
    return reduce(np.kron, mats)


def dense_spin_H(lat):
    """H of the J1-J2 model as a 2^N x 2^N matrix, site 0 most significant."""
    N = lat.N
    H = np.zeros((2 ** N, 2 ** N))
    pairs = [(lat.site(*a), lat.site(*b), lat.J1) for a, b in lat.bonds_h() + lat.bonds_v()]
    pairs += [(lat.site(*a), lat.site(*b), lat.J2) for a, b in lat.bonds_d()]
    for i, j, J in pairs:
        if J == 0.0:
            continue
        H += J * _embed({i: _SZ, j: _SZ}, N, 2, _I2)
        H += 0.5 * J * _embed({i: _SP, j: _SM}, N, 2, _I2)
        H += 0.5 * J * _embed({i: _SM, j: _SP}, N, 2, _I2)
    return H


def _fermion_spin_dot(cs, i, j):
    """S_i.S_j from the Jordan-Wigner mode operators: S^z = (n_up - n_dn)/2,
    S^+ = c^dag_up c_dn, S^- its transpose."""
    def spin_ops(k):
        cu, cd = cs[2 * k], cs[2 * k + 1]
        sz = 0.5 * (cu.T @ cu - cd.T @ cd)
        sp = cu.T @ cd
        return sz, sp
    szi, spi = spin_ops(i)
    szj, spj = spin_ops(j)
    return szi @ szj + 0.5 * (spi @ spj.T + spi.T @ spj)


def dense_hubbard_H(lat):
    """Hubbard H as a 4^N x 4^N matrix in the occupation basis.  Modes are
    ordered (site 0 up, site 0 down, site 1 up, ...); the matrix index of a
    state is read with site 0 most significant and, within a site, the digit
    s = n_up + 2 n_dn.  Fermion operators are built as Jordan-Wigner products
    sigma^z ... sigma^z a over the 2N modes, then mapped to that basis."""
    N = lat.N
    M = 2 * N
    a = np.array([[0.0, 1.0], [0.0, 0.0]])   # annihilator in mode basis (|0>, |1>)
    zz = np.diag([1.0, -1.0])
    i2 = np.eye(2)

    def ann(m):
        return reduce(np.kron, [zz] * m + [a] + [i2] * (M - m - 1))

    cs = [ann(m) for m in range(M)]
    dimf = 2 ** M
    Hf = np.zeros((dimf, dimf))
    for i, j, _ in hubbard_pairs(lat):
        for sg in (0, 1):
            ci, cj = cs[2 * i + sg], cs[2 * j + sg]
            Hf += -lat.t * (ci.T @ cj + cj.T @ ci)
    for i in range(N):
        nu = cs[2 * i].T @ cs[2 * i]
        nd = cs[2 * i + 1].T @ cs[2 * i + 1]
        Hf += lat.U * nu @ nd - lat.mu * (nu + nd)
    if lat.J2 != 0.0:
        for i, j in ((lat.site(*a), lat.site(*b)) for a, b in lat.bonds_d()):
            Hf += lat.J2 * _fermion_spin_dot(cs, i, j)
    # mode-basis index: mode 0 most significant bit.  Map to digit basis.
    perm = np.zeros(dimf, dtype=np.int64)
    for idx in range(dimf):
        occ = [(idx >> (M - 1 - m)) & 1 for m in range(M)]
        dig = 0
        for k in range(N):
            dig = dig * 4 + (occ[2 * k] + 2 * occ[2 * k + 1])
        perm[dig] = idx
    return Hf[np.ix_(perm, perm)]


def dense_H(lat):
    if lat.model == MODEL_HEISENBERG:
        return dense_spin_H(lat)
    return dense_hubbard_H(lat)
