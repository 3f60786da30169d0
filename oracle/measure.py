"""Per-sample quantities of the Monte Carlo estimators (Method section,
Eqs. (8)-(9)): log|psi|, sign, the local energy E_loc and the log-derivative
row O, all from boundary-MPS strips.

Readings (the paper does not say which contraction supplies each number):
  * log|psi| := log|rho_{L1-1}(S)|, the top-down amplitude
    <top[L1-2] | M_{L1-1}>;
  * a ratio rho(S')/rho(S) for a term acting inside row r uses the one-row
    strip rho_r; a term that touches rows r and r+1 uses the two-row strip
    rho_{r,r+1}; numerator and denominator share the same boundaries;
  * O for the entries of site (r, c) is d rho_r / d T_{rc}[S_rc] / rho_r with
    top[r-1] and bot[r+1] held fixed (exact: neither depends on row r); every
    other slice of site (r, c) has O = 0, so a row stores one block per site.
"""
from __future__ import annotations

import math

import numpy as np

from . import bmps
from .hamiltonian import local_energy


class ZeroAmplitude(ArithmeticError):
    pass


def evaluate(lat, theta, S, chi, tops=None, bots=None, want_O=True):
    """Dict with log_abs, sign, e_loc and (optionally) the O row."""
    S = np.asarray(S, dtype=np.int64).reshape(lat.N)
    L1 = lat.L1
    if tops is None:
        tops = bmps.top_boundaries(lat, theta, S, chi)
    if bots is None:
        bots = bmps.bot_boundaries(lat, theta, S, chi)
    W = [lat.row_slices(theta, S, r) for r in range(L1)]
    # tops[r] is top[r-1]; bots[r] is bot[r]
    rho1 = [bmps.strip1(tops[r][0], W[r], bots[r + 1][0]) for r in range(L1)]
    rho2 = [bmps.strip2(tops[r][0], W[r], W[r + 1], bots[r + 2][0]) for r in range(L1 - 1)]
    last = rho1[L1 - 1]
    if last == 0.0 or any(v == 0.0 for v in rho1) or any(v == 0.0 for v in rho2):
        raise ZeroAmplitude("configuration has zero strip amplitude")
    log_abs = tops[L1 - 1][1] + math.log(abs(last))
    sign = 1 if last > 0 else -1

    def ratio(S2, info):
        i, j = info[0], info[1]
        ri, rj = i // lat.L2, j // lat.L2
        r = min(ri, rj)
        if ri == rj:
            W2 = lat.row_slices(theta, S2, r)
            return bmps.strip1(tops[r][0], W2, bots[r + 1][0]) / rho1[r]
        W2a = lat.row_slices(theta, S2, r)
        W2b = lat.row_slices(theta, S2, r + 1)
        return bmps.strip2(tops[r][0], W2a, W2b, bots[r + 2][0]) / rho2[r]

    e_loc = local_energy(lat, S, ratio)
    out = {"log_abs": log_abs, "sign": sign, "e_loc": e_loc}
    if want_O:
        off, nnz = lat.orow_offsets()
        O = np.zeros(nnz)
        for r in range(L1):
            for c in range(lat.L2):
                env = bmps.strip1_env(tops[r][0], W[r], bots[r + 1][0], c)
                o = off[lat.site(r, c)]
                O[o:o + env.size] = env.reshape(-1) / rho1[r]
        out["O"] = O
    return out


def evaluate_batch(lat, theta, configs, chi, want_O=True):
    """Evaluate every row of `configs` ([n, N])."""
    res = [evaluate(lat, theta, S, chi, want_O=want_O) for S in np.asarray(configs)]
    out = {
        "log_abs": np.array([x["log_abs"] for x in res]),
        "sign": np.array([x["sign"] for x in res], dtype=np.int8),
        "e_loc": np.array([x["e_loc"] for x in res]),
    }
    if want_O:
        out["O"] = np.stack([x["O"] for x in res])
    return out


def expand_O(lat, S, O_row):
    """The full log-derivative vector (length N_p) of one sample."""
    S = np.asarray(S, dtype=np.int64).reshape(lat.N)
    poff, n_p = lat.param_offsets()
    ooff, _ = lat.orow_offsets()
    full = np.zeros(n_p)
    for r in range(lat.L1):
        for c in range(lat.L2):
            i = lat.site(r, c)
            bs = lat.block_size(r, c)
            start = poff[i] + int(S[i]) * bs
            full[start:start + bs] = O_row[ooff[i]:ooff[i] + bs]
    return full
