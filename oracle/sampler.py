"""Metropolis sweep over configurations S = (s, s') (Method section: the
state is sampled by Markov-chain Monte Carlo with weight |rho_theta(S)|^2;
Appendix A: with weight |rho|^alpha, alpha = 1, for the reweighted form).

The paper fixes neither the proposal set nor the order.  Reading taken:
for each row r = 0..L1-1 in turn, with top[r-1] built from the rows already
swept and bot[r+1] from the configuration at the start of the sweep:
  1. horizontal bonds c = 0..L2-2: exchange the ket digits, then the bra
     digits, of (r,c) and (r,c+1) (Hubbard: per species, up then down, ket
     then bra);  ratio from the one-row strip rho_r;
  2. site moves c = 0..L2-1: spin (s,s) -> (1-s, 1-s); Hubbard: per species,
     toggle n_sigma of ket and bra together when they agree;  ratio rho_r;
  3. if r < L1-1, vertical bonds c = 0..L2-1, exchanges between (r,c) and
     (r+1,c) as in 1; ratio from the two-row strip rho_{r,r+1};
  4. top[r] = C_chi(top[r-1] o M_r).
A proposal that would not change S is skipped, but still owns its slot.
Accept iff u < min(1, |R|^alpha), R = rho(S')/rho(S), u the slot's uniform.
Every proposal is an involution of the local state, hence symmetric.
"""
from __future__ import annotations

import numpy as np

from . import bmps
from .lattice import MODEL_HEISENBERG
from .philox import uniform

MOVE_H, MOVE_SITE, MOVE_V = 0, 1, 2


def _bond_proposal(lat, S, a, b, k):
    """Exchange proposal number k on bond (a, b) (flat site indices)."""
    if lat.model == MODEL_HEISENBERG:
        side = k
        sa = lat.ket(S[a]) if side == 0 else lat.bra(S[a])
        sb = lat.ket(S[b]) if side == 0 else lat.bra(S[b])
        if sa == sb:
            return None
        S2 = S.copy()
        if side == 0:
            S2[a] = lat.merge(sb, lat.bra(S[a]))
            S2[b] = lat.merge(sa, lat.bra(S[b]))
        else:
            S2[a] = lat.merge(lat.ket(S[a]), sb)
            S2[b] = lat.merge(lat.ket(S[b]), sa)
        return S2
    # Hubbard: k = 2 * side + sigma  -> order: (ket,up) (ket,dn) (bra,up) (bra,dn)
    side, sg = k // 2, k % 2
    da = lat.ket(S[a]) if side == 0 else lat.bra(S[a])
    db = lat.ket(S[b]) if side == 0 else lat.bra(S[b])
    na, nb = (da >> sg) & 1, (db >> sg) & 1
    if na == nb:
        return None
    da2, db2 = da ^ (1 << sg), db ^ (1 << sg)
    S2 = S.copy()
    if side == 0:
        S2[a] = lat.merge(da2, lat.bra(S[a]))
        S2[b] = lat.merge(db2, lat.bra(S[b]))
    else:
        S2[a] = lat.merge(lat.ket(S[a]), da2)
        S2[b] = lat.merge(lat.ket(S[b]), db2)
    return S2


def _site_proposal(lat, S, i, k):
    s, sp = lat.ket(S[i]), lat.bra(S[i])
    if lat.model == MODEL_HEISENBERG:
        if s != sp:
            return None
        S2 = S.copy()
        S2[i] = lat.merge(1 - s, 1 - sp)
        return S2
    sg = k
    if ((s >> sg) & 1) != ((sp >> sg) & 1):
        return None
    S2 = S.copy()
    S2[i] = lat.merge(s ^ (1 << sg), sp ^ (1 << sg))
    return S2


def accept(u, R, alpha):
    """Metropolis decision with the positional uniform u."""
    w = R * R if alpha == 2 else abs(R)
    return u < min(1.0, w), abs(u - min(1.0, w))


def sweep(lat, theta, S, chi, seed, chain, gsweep, alpha=2, bots=None, tie_tol=1e-12):
    """One sweep of one chain.  Returns dict(S, n_accept[3], n_prop[3], tops,
    near_ties) where tops[r] = top[r-1] for the final configuration."""
    S = np.array(S, dtype=np.int64).reshape(lat.N).copy()
    L1, L2 = lat.L1, lat.L2
    if bots is None:
        bots = bmps.bot_boundaries(lat, theta, S, chi)
    tops = [bmps.trivial(L2)]
    slot = 0
    n_acc = [0, 0, 0]
    n_prop = [0, 0, 0]
    ties = []

    def try_move(S2, kind, rho_fn, u):
        nonlocal S
        R = rho_fn(S2) / rho_fn(S)
        ok, gap = accept(u, R, alpha)
        n_prop[kind] += 1
        if gap <= tie_tol:
            ties.append((chain, gsweep, slot, R, u))
        if ok:
            S = S2
            n_acc[kind] += 1

    for r in range(L1):
        top = tops[-1][0]
        bot1 = bots[r + 1][0]

        def rho_row(X, r=r, top=top, bot1=bot1):
            return bmps.strip1(top, lat.row_slices(theta, X, r), bot1)

        for c in range(L2 - 1):
            a, b = lat.site(r, c), lat.site(r, c + 1)
            for k in range(lat.n_bond_moves()):
                u = uniform(seed, chain, gsweep, slot)
                S2 = _bond_proposal(lat, S, a, b, k)
                if S2 is not None:
                    try_move(S2, MOVE_H, rho_row, u)
                slot += 1
        for c in range(L2):
            i = lat.site(r, c)
            for k in range(lat.n_site_moves()):
                u = uniform(seed, chain, gsweep, slot)
                S2 = _site_proposal(lat, S, i, k)
                if S2 is not None:
                    try_move(S2, MOVE_SITE, rho_row, u)
                slot += 1
        if r < L1 - 1:
            bot2 = bots[r + 2][0]

            def rho_two(X, r=r, top=top, bot2=bot2):
                return bmps.strip2(top, lat.row_slices(theta, X, r),
                                   lat.row_slices(theta, X, r + 1), bot2)

            for c in range(L2):
                a, b = lat.site(r, c), lat.site(r + 1, c)
                for k in range(lat.n_bond_moves()):
                    u = uniform(seed, chain, gsweep, slot)
                    S2 = _bond_proposal(lat, S, a, b, k)
                    if S2 is not None:
                        try_move(S2, MOVE_V, rho_two, u)
                    slot += 1
        A, ls = tops[-1]
        Ac, dl = bmps.compress(bmps.absorb_top(A, lat.row_slices(theta, S, r)), chi)
        tops.append((Ac, ls + dl))
    assert slot == lat.n_slots()
    return {"S": S, "n_accept": n_acc, "n_prop": n_prop, "tops": tops, "near_ties": ties}


def run_chain(lat, theta, S0, chi, seed, chain, gsweep0, n_sweeps, alpha=2):
    """n_sweeps consecutive sweeps; returns the list of per-sweep results."""
    out = []
    S = np.array(S0, dtype=np.int64)
    for k in range(n_sweeps):
        res = sweep(lat, theta, S, chi, seed, chain, gsweep0 + k, alpha=alpha)
        S = res["S"]
        out.append(res)
    return out
