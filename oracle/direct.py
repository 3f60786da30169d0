"""Direct (autoregressive) sampling of the vectorised PEPS (Appendix A,
Eqs. A2-A7): configurations are drawn site by site, row-major, each site
from its conditional probability given the sites already drawn,
    p_2c(S_i | S_<i) = sum_{S_>i} |rho(S)|^2 / sum_{S_>=i} |rho(S)|^2,
so that p_2(S) = prod_i p_2c = |rho(S)|^2 / Z; or, reweighted,
    p_4c(S_i | S_<i) proportional to b(S_i) sqrt(p_2c(S_i | S_<i)),
with b = 1 on off-diagonal digit pairs (s != s') and b = b_diag on diagonal
ones.  Averages take the weights r = |rho(S)|^2 / p(S) (Eq. A7; the same
weights make the p_2 estimator exact when the marginals are approximate).

The paper leaves the algorithm of the marginals to its reference; reading
taken here (everything a plain, slow reference):

  * the double-layer network sum_S rho(S)^2 is a PEPS without physical leg
    whose site tensors are E_i = sum_S T_i[S] (x) T_i[S] (bond dimension
    D^2, index (x, x') with x' fastest);
  * its bottom boundaries bdl[r] (rows r..L1-1) come from the same C_chi as
    the single-layer ones, with boundary dimension chi_dl;
  * the rows above the current one are drawn, so their double layer is the
    single-layer top boundary paired with itself, top (x) top;
  * the marginal of site (r, c) for digit x is the one-row strip
    <top (x) top | P(S_r,0) .. P(S_r,c-1) P(x) E_r,c+1 .. E_r,L2-1 | bdl[r+1]>,
    P(S) = T[S] (x) T[S]; a negative value (truncation) counts as 0;
  * site i = r L2 + c takes the uniform u of Philox4x64-10 with counter
    (chain, draw, i, 3) and key (seed, 0), and the digit x is the first
    whose running sum of probabilities (in digit order) exceeds u (the
    last digit of nonzero probability if none does);
  * after row r, top[r] = C_chi(top[r-1] o row r) on the drawn digits;
  * b_diag (the paper: "updated every gradient step" so that diagonal
    configurations are at most half of the samples) is multiplied after a
    step by (1/2 / f)^(1/N), f the fraction of drawn configurations with
    s = s' on every site, and capped at 1 (f = 0 counts as f = 1/4).

Test infrastructure only: nothing on the product path imports this package.
"""
from __future__ import annotations

import math

import numpy as np

from . import bmps, philox


def pair(T):
    """T[l, u, r, d] (x) T[l', u', r', d'] as one tensor over merged legs."""
    l, u, r, d = T.shape
    return np.einsum("lurd,LURD->lLuUrRdD", T, T).reshape(l * l, u * u, r * r, d * d)


def double_layer_row(lat, theta, r):
    """E_c = sum_S T_{rc}[S] (x) T_{rc}[S] for the columns of row r."""
    row = []
    for c in range(lat.L2):
        Ts = lat.site_tensor(theta, r, c)
        row.append(sum(pair(Ts[S]) for S in range(lat.d2)))
    return row


def double_layer_bottoms(lat, theta, chi_dl):
    """[bdl[0], ..., bdl[L1]]: bdl[r] covers rows r..L1-1 of the double
    layer, bdl[L1] is trivial."""
    bots = [None] * (lat.L1 + 1)
    bots[lat.L1] = bmps.trivial(lat.L2)
    for r in range(lat.L1 - 1, -1, -1):
        A, ls = bots[r + 1]
        Ac, dl = bmps.compress(bmps.absorb_bot(A, double_layer_row(lat, theta, r)), chi_dl)
        bots[r] = (Ac, ls + dl)
    return bots


def double_top(top):
    """A single-layer boundary paired with itself: bond dimensions squared."""
    out = []
    for A in top:
        a, u, b = A.shape
        out.append(np.einsum("aub,AUB->aAuUbB", A, A).reshape(a * a, u * u, b * b))
    return out


def site_weights(lat, theta, S, r, c, top_dbl, bdl_row):
    """Unnormalised marginals q(x), x in [0, d^2), of site (r, c) given the
    digits S of the sites before it (row-major)."""
    E = double_layer_row(lat, theta, r)
    q = np.zeros(lat.d2)
    for x in range(lat.d2):
        W = []
        for cc in range(lat.L2):
            if cc < c:
                W.append(pair(lat.site_tensor(theta, r, cc)[int(S[r * lat.L2 + cc])]))
            elif cc == c:
                W.append(pair(lat.site_tensor(theta, r, cc)[x]))
            else:
                W.append(E[cc])
        q[x] = max(bmps.strip1(top_dbl, W, bdl_row), 0.0)
    return q


def site_probs(lat, q, reweight, b_diag):
    """p_2c from q, or the reweighted p_4c (Eqs. A3, A5, A6)."""
    tot = q.sum()
    if not tot > 0.0:
        return None
    p2 = q / tot
    if not reweight:
        return p2
    b = np.array([1.0 if lat.ket(x) != lat.bra(x) else b_diag for x in range(lat.d2)])
    w = b * np.sqrt(p2)
    return w / w.sum()


def pick(p, u):
    """First digit whose running sum exceeds u; else the last one of
    nonzero probability.  Also the distance of u to the nearest running sum
    (a near-tie when tiny)."""
    cum, gap = 0.0, math.inf
    last = int(np.nonzero(p > 0.0)[0][-1])
    for x in range(len(p)):
        cum += p[x]
        gap = min(gap, abs(u - cum))
        if u < cum:
            return x, gap
    return last, gap


def sample(lat, theta, chi, chi_dl, seed, chain, draw, reweight=False, b_diag=1.0, bdl=None):
    """One configuration.  Returns dict(S, log_p, gap): log_p is the log of
    the probability the sampler gave S (the product of the conditionals it
    used), gap the smallest distance of a uniform to a running sum."""
    if bdl is None:
        bdl = double_layer_bottoms(lat, theta, chi_dl)
    S = np.zeros(lat.N, dtype=np.int64)
    log_p, gap = 0.0, math.inf
    top = bmps.trivial(lat.L2)
    for r in range(lat.L1):
        tdbl = double_top(top[0])
        for c in range(lat.L2):
            i = r * lat.L2 + c
            p = site_probs(lat, site_weights(lat, theta, S, r, c, tdbl, bdl[r + 1][0]), reweight, b_diag)
            if p is None:
                return {"S": S, "log_p": -math.inf, "gap": 0.0}
            x, g = pick(p, philox.uniform(seed, chain, draw, i, stream=3))
            S[i] = x
            log_p += math.log(p[x])
            gap = min(gap, g)
        A, ls = top
        Ac, dl = bmps.compress(bmps.absorb_top(A, lat.row_slices(theta, S, r)), chi)
        top = (Ac, ls + dl)
    return {"S": S, "log_p": log_p, "gap": gap}


def log_prob(lat, theta, S, chi, chi_dl, reweight=False, b_diag=1.0, bdl=None):
    """log of the probability the sampler assigns to a given configuration
    (the product of its conditionals along S)."""
    if bdl is None:
        bdl = double_layer_bottoms(lat, theta, chi_dl)
    S = np.asarray(S, dtype=np.int64).reshape(lat.N)
    lp = 0.0
    top = bmps.trivial(lat.L2)
    for r in range(lat.L1):
        tdbl = double_top(top[0])
        for c in range(lat.L2):
            p = site_probs(lat, site_weights(lat, theta, S, r, c, tdbl, bdl[r + 1][0]), reweight, b_diag)
            if p is None or p[S[r * lat.L2 + c]] == 0.0:
                return -math.inf
            lp += math.log(p[S[r * lat.L2 + c]])
        A, ls = top
        Ac, dl = bmps.compress(bmps.absorb_top(A, lat.row_slices(theta, S, r)), chi)
        top = (Ac, ls + dl)
    return lp


def update_b(lat, b_diag, configs):
    """The dynamic diagonal weight after a step whose drawn configurations
    are `configs` [n, N] (reading in the module docstring)."""
    cfg = np.asarray(configs)
    diag = np.all(cfg // lat.d == cfg % lat.d, axis=1)
    f = float(diag.mean()) if diag.size else 0.25
    if f == 0.0:
        f = 0.25
    return min(1.0, b_diag * (0.5 / f) ** (1.0 / lat.N))
