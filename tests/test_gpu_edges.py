"""Edge cases of the device path against the oracle: the smallest lattice,
bond dimension 1 (product states), boundary dimension 1 (every cut truncated
to one value), the widest row (L2 = 32) and the largest site count
(L1 L2 = 256); empty batches for every entry point (no-ops); and the exact
beta = 0 state, whose truncations are fully degenerate, against closed forms.
Bars as in the other FP64 parity tests."""
import sys

import numpy as np
import pytest

import synth
from closed_forms import identity_closed_forms, identity_closed_forms_hubbard
from oracle import measure, sampler
from oracle.lattice import Lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


CASES = [
    (2, 2, 1, 1),      # smallest lattice, product state
    (2, 2, 2, 1),      # chi = 1: every cut truncated to its largest value
    (2, 3, 1, 4),      # D = 1 with chi above every bond
    (2, 32, 2, 4),     # widest row
    (16, 16, 2, 4),    # largest number of sites
    (8, 32, 2, 3),     # largest number of sites with the widest row, truncating
]


@pytest.mark.parametrize("L1,L2,D,chi", CASES)
def test_edge_shapes_match_oracle(L1, L2, D, chi):
    dev = _dev()
    import paper_2409_05285_amd as p
    print("[case] edge", L1, L2, D, chi, flush=True)
    sys.stdout.flush()
    lat = Lattice(L1, L2, D=D, chi=chi)
    desc = p.Desc(L1, L2, D, chi)
    th = synth.theta_random_unit(L1, L2, D, 2, seed=5)
    cfg = synth.configs_sector(2, lat.N, 2, seed=6)
    theta_d = torch.tensor(th, device=dev)
    la, sg, el, st = p.peps_eval_batch(desc, theta_d, torch.tensor(cfg, device=dev))
    O, _, st2 = p.peps_grad_batch(desc, theta_d, torch.tensor(cfg, device=dev))
    torch.cuda.synchronize()
    assert p.check(st) == 0 and p.check(st2) == 0
    ref = measure.evaluate_batch(lat, th, cfg, chi)
    la, sg, el, O = (x.cpu().numpy() for x in (la, sg, el, O))
    assert np.all(np.abs(la - ref["log_abs"]) <= 1e-10 * np.maximum(1.0, np.abs(ref["log_abs"])))
    assert np.array_equal(sg, ref["sign"])
    emag = max(np.abs(ref["e_loc"]).mean(), 1e-300)
    assert np.all(np.abs(el - ref["e_loc"]) <= 1e-10 * np.maximum(np.abs(ref["e_loc"]), emag))
    assert np.all(np.abs(O - ref["O"]) <= 1e-9 * np.maximum(1.0, np.abs(ref["O"])))
    # one sweep, bit-exact
    cfg0 = synth.configs_diagonal(2, lat.N, 2, seed=7)
    cfg_d = torch.tensor(cfg0, device=dev)
    res = p.peps_sample_sweep(desc, theta_d, cfg_d, 11, 0, 1)
    torch.cuda.synchronize()
    assert p.check(res["status"]) == 0
    got = cfg_d.cpu().numpy()
    for ch in range(2):
        r = sampler.sweep(lat, th, cfg0[ch].astype(np.int64), chi, 11, ch, 0)
        if r["near_ties"]:
            continue
        assert np.array_equal(got[ch], r["S"].astype(np.uint8)), ch


def test_empty_batches_are_noops():
    dev = _dev()
    import paper_2409_05285_amd as p
    desc = p.Desc(4, 4, 2, 4)
    theta = torch.tensor(synth.theta_random_unit(4, 4, 2, 2, seed=1), device=dev)
    empty = torch.zeros((0, 16), dtype=torch.uint8, device=dev)
    la, sg, el, st = p.peps_eval_batch(desc, theta, empty)
    O, la2, st2 = p.peps_grad_batch(desc, theta, empty)
    res = p.peps_sample_sweep(desc, theta, empty, 1, 0, 1)
    obs = p.peps_observables_batch(desc, empty)
    torch.cuda.synchronize()
    assert la.shape == (0,) and O.shape == (0, p.peps_orow_count(desc)) and obs.shape == (0, 4)
    assert res["O"].shape == (1, 0, p.peps_orow_count(desc))
    assert p.check(st) == 0 and p.check(st2) == 0 and p.check(res["status"]) == 0
    # zero sweeps on a non-empty batch leave the configurations untouched
    cfg = torch.tensor(synth.configs_diagonal(3, 16, 2, seed=2), device=dev)
    before = cfg.clone()
    p.peps_sample_sweep(desc, theta, cfg, 1, 0, 0, measure=False)
    torch.cuda.synchronize()
    assert torch.equal(cfg, before)


@pytest.mark.parametrize("mixed", [False, True])
def test_beta0_identity_closed_forms_hubbard(mixed):
    """The exact beta = 0 state of the Hubbard model (d^2 = 16, 6 x 6, D = 4,
    chi = 16, U = 8, mu = 4, J2 = 0.6) against its closed forms."""
    dev = _dev()
    import paper_2409_05285_amd as p
    print("[case] beta0 identity hubbard", mixed, flush=True)
    sys.stdout.flush()
    L1 = L2 = 6
    desc = p.Desc(L1, L2, 4, 16, d=4, model=p.MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0, J2=0.6,
                  precision=p.PREC_MIXED if mixed else p.PREC_FP64)
    th = torch.tensor(synth.theta_identity(L1, L2, 4, 4), device=dev)
    cfg = synth.configs_diagonal(32, L1 * L2, 4, seed=58)
    cfg_d = torch.tensor(cfg, device=dev)
    la, sg, el, st = p.peps_eval_batch(desc, th, cfg_d)
    O, la2, st2 = p.peps_grad_batch(desc, th, cfg_d)
    torch.cuda.synchronize()
    assert p.check(st) == 0 and p.check(st2) == 0
    e_ref, o_ref = identity_closed_forms_hubbard(L1, L2, 4, 8.0, 4.0, 0.6, cfg)
    la, sg, el, la2, O = la.cpu().numpy(), sg.cpu().numpy(), el.cpu().numpy(), la2.cpu().numpy(), O.cpu().numpy()
    tol = 1e-4 if mixed else 1e-10
    assert np.all(np.abs(la) <= tol) and np.all(np.abs(la2) <= tol)
    assert np.all(sg == 1)
    assert np.all(np.abs(el - e_ref) <= tol * np.maximum(1.0, np.abs(e_ref))), np.abs(el - e_ref).max()
    assert np.all(np.abs(O - o_ref[None, :]) <= (1e-4 if mixed else 1e-9)), np.abs(O - o_ref[None, :]).max()


@pytest.mark.parametrize("L1,L2,D,chi,J2,mixed", [(8, 8, 4, 16, 0.0, False), (8, 8, 4, 16, 0.0, True),
                                                  (4, 4, 6, 36, 0.5, False), (4, 4, 6, 36, 0.5, True)])
def test_beta0_identity_closed_forms(L1, L2, D, chi, J2, mixed):
    """The exact beta = 0 state, where every truncated cut has one nonzero
    singular value and the rest are exactly zero (the fully degenerate case
    of the truncation), against its closed forms: log|psi| = 0, sign +1,
    E_loc = 2 H_ss and the O rows, on the register-resident (chi D = 64) and
    the workspace (chi D = 216) compression paths."""
    dev = _dev()
    import paper_2409_05285_amd as p
    print("[case] beta0 identity", L1, L2, D, chi, J2, mixed, flush=True)
    sys.stdout.flush()
    desc = p.Desc(L1, L2, D, chi, J2=J2, precision=p.PREC_MIXED if mixed else p.PREC_FP64)
    th = torch.tensor(synth.theta_identity(L1, L2, D, 2), device=dev)
    cfg = synth.configs_diagonal(32, L1 * L2, 2, seed=57)
    cfg_d = torch.tensor(cfg, device=dev)
    la, sg, el, st = p.peps_eval_batch(desc, th, cfg_d)
    O, la2, st2 = p.peps_grad_batch(desc, th, cfg_d)
    torch.cuda.synchronize()
    assert p.check(st) == 0 and p.check(st2) == 0
    e_ref, o_ref = identity_closed_forms(L1, L2, D, 1.0, J2, cfg)
    la, sg, el, la2, O = la.cpu().numpy(), sg.cpu().numpy(), el.cpu().numpy(), la2.cpu().numpy(), O.cpu().numpy()
    tol = 1e-4 if mixed else 1e-10
    assert np.all(np.abs(la) <= tol) and np.all(np.abs(la2) <= tol), (np.abs(la).max(), np.abs(la2).max())
    assert np.all(sg == 1)
    assert np.all(np.abs(el - e_ref) <= tol * np.maximum(1.0, np.abs(e_ref))), np.abs(el - e_ref).max()
    assert np.all(np.abs(O - o_ref[None, :]) <= (1e-4 if mixed else 1e-9)), np.abs(O - o_ref[None, :]).max()


@pytest.mark.parametrize("weighted", [False, True])
def test_beta0_sr_step_closed_form(weighted):
    """SR at the exact beta = 0 state from closed-form inputs (8 x 8, D = 4,
    512 diagonal samples): a sample's O row is 1 on the zero-leg entry of
    its own slice (s_j, s_j) at every site j, so only the 2 N indicator
    parameters are active.  There g_k = sum_i p_i [S_j(i) = S] (E_i - Ebar)
    (the sample covariance of a spin with the energy: zero in expectation,
    as the exact gradient at the identity is, but not for a finite sample),
    the metric is the covariance of the indicators, and
    (S + eps 1) dtheta = -tau g (Eqs. 5-7) is solved densely on the host;
    every other entry of g and dtheta is zero.  With weights, all |rho| = 1
    as the alpha = 1 reweighting gives there."""
    dev = _dev()
    import paper_2409_05285_amd as p
    print("[case] beta0 SR closed form, weighted", weighted, flush=True)
    sys.stdout.flush()
    L1 = L2 = 8
    D, N, tau, eps = 4, 64, 0.02, 1e-4
    desc = p.Desc(L1, L2, D, 16, alpha=1 if weighted else 2)
    cfg = synth.configs_diagonal(512, N, 2, seed=59)
    n = cfg.shape[0]
    e_ref, o_ref = identity_closed_forms(L1, L2, D, 1.0, 0.0, cfg)
    O = torch.tensor(np.ascontiguousarray(np.tile(o_ref, (n, 1))), device=dev)
    E = torch.tensor(e_ref, device=dev)
    w = torch.ones(n, dtype=torch.float64, device=dev) if weighted else None
    dth, g, stats, st = p.sr_cg_solve(desc, torch.tensor(cfg, device=dev), O, E, tau, eps, 400, 1e-12, weights=w)
    torch.cuda.synchronize()
    assert p.check(st) in (0, 1)   # 1: CG stopped at max_iter (reported, not an error)
    g, dth, stats = g.cpu().numpy(), dth.cpu().numpy(), stats.cpu().numpy()
    # parameter index of the zero-leg entry of slice S at site j: site-major
    # blocks of d^2 slices, each slice the product of the site's leg dims
    off, bsz = [], []
    po = 0
    for r in range(L1):
        for c in range(L2):
            b = (1 if c == 0 else D) * (1 if r == 0 else D) * (1 if c == L2 - 1 else D) * (1 if r == L1 - 1 else D)
            off.append(po)
            bsz.append(b)
            po += 4 * b
    assert po == g.size
    X = np.zeros((n, 2 * N))                     # indicator of (s_j = 0) and (s_j = 1)
    idx = np.zeros(2 * N, dtype=np.int64)
    for j in range(N):
        for s_ in range(2):
            X[:, 2 * j + s_] = (cfg[:, j] // 2 == s_)
            idx[2 * j + s_] = off[j] + (3 * s_) * bsz[j]
    pw = np.full(n, 1.0 / n)
    ebar = pw @ e_ref
    g_act = X.T @ (pw * (e_ref - ebar))
    xbar = pw @ X
    S = (X * pw[:, None]).T @ X - np.outer(xbar, xbar)
    d_act = np.linalg.solve(S + eps * np.eye(2 * N), -tau * g_act)
    g_ref = np.zeros(g.size)
    g_ref[idx] = g_act
    d_ref = np.zeros(g.size)
    d_ref[idx] = d_act
    assert abs(stats[0] - ebar) <= 1e-12 * max(1.0, abs(ebar))
    assert np.abs(g - g_ref).max() <= 1e-12 * max(1.0, np.abs(g_ref).max()), np.abs(g - g_ref).max()
    assert np.abs(dth - d_ref).max() <= 1e-8 * np.abs(d_ref).max(), (np.abs(dth - d_ref).max(), np.abs(d_ref).max())
