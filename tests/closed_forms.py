"""Closed forms of the exact beta = 0 state |I> (every site's slice (s, s)
is 1 at bond index 0, all else 0; Method section, the identity as the
infinite-temperature state), used by the CPU pin against the oracle and by
the device tests: written from the definitions alone, independent of both
the oracle and the library."""
import numpy as np


def identity_closed_forms(L1, L2, D, J1, J2, cfg):
    """beta = 0 state |I> (every site's slice (s, s) is 1 at bond index 0):
    for a diagonal configuration rho = 1, and every off-diagonal term of
    H (x) I + I (x) H^T leads to a configuration with s != s', where rho = 0,
    so E_loc = 2 H_ss = 2 sum_<ij> J Sz_i Sz_j over nearest and next-nearest
    neighbours; the derivative of rho by the slice entry with every leg at 0
    is 1 and by every other entry 0 (method section, Eqs. 4, 8 and 9)."""
    sz = 0.5 - (cfg // 2).astype(np.float64)          # digit 0 = spin up
    sz = sz.reshape(cfg.shape[0], L1, L2)
    h = J1 * ((sz[:, :, :-1] * sz[:, :, 1:]).sum(axis=(1, 2)) + (sz[:, :-1, :] * sz[:, 1:, :]).sum(axis=(1, 2)))
    h += J2 * ((sz[:, :-1, :-1] * sz[:, 1:, 1:]).sum(axis=(1, 2)) + (sz[:, :-1, 1:] * sz[:, 1:, :-1]).sum(axis=(1, 2)))
    row = []
    for r in range(L1):
        for c in range(L2):
            n = (1 if c == 0 else D) * (1 if r == 0 else D) * (1 if c == L2 - 1 else D) * (1 if r == L1 - 1 else D)
            blk = np.zeros(n)
            blk[0] = 1.0
            row.append(blk)
    return 2.0 * h, np.concatenate(row)


def identity_closed_forms_hubbard(L1, L2, D, U, mu, J2, cfg):
    """The same for the Hubbard model (digit s = n_up + 2 n_dn): the
    diagonal of H is U n_up n_dn - mu (n_up + n_dn) per site plus
    J2 Sz_i Sz_j, Sz = (n_up - n_dn) / 2, on next-nearest neighbours."""
    s = (cfg // 4).reshape(cfg.shape[0], L1, L2)
    nu, nd = (s & 1).astype(np.float64), ((s >> 1) & 1).astype(np.float64)
    sz = 0.5 * (nu - nd)
    h = (U * nu * nd - mu * (nu + nd)).sum(axis=(1, 2))
    h += J2 * ((sz[:, :-1, :-1] * sz[:, 1:, 1:]).sum(axis=(1, 2)) + (sz[:, :-1, 1:] * sz[:, 1:, :-1]).sum(axis=(1, 2)))
    _, o = identity_closed_forms(L1, L2, D, 0.0, 0.0, cfg)
    return 2.0 * h, o
