"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Tolerances (FP64 path): |d log|psi|| <= 1e-10 max(1, |log|psi||);
|d E_loc| <= 1e-10 max(|E_loc|, mean|E|); |d O| <= 1e-9 max(1, |O|);
configurations, accept counts and signs bit-exact (except after a logged
near-tie of the Metropolis test, |u - min(1,|R|^2)| <= 1e-12).

Mixed precision (FP32 strip contractions, FP64 truncation and reductions):
log|psi| and E_loc within 1e-4 relative (same normalisations as above), O
within 1e-4 of the row's largest magnitude, signs exact; sampled
configurations and accept counts bit-exact for every chain whose Metropolis
tests all stay 1e-4 away from a tie.
"""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import measure, sampler, sr
from oracle.lattice import Lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _setup(L1, L2, D, chi, J2=0.0, theta="random", seed=7, mixed=False, scale=1.0):
    import paper_2409_05285_amd as p
    lat = Lattice(L1, L2, D=D, chi=chi, J1=1.0, J2=J2)
    desc = p.Desc(L1, L2, D, chi, J1=1.0, J2=J2, precision=p.PREC_MIXED if mixed else p.PREC_FP64)
    if theta == "random":
        th = synth.theta_random_unit(L1, L2, D, 2, seed=seed)
    else:
        th = synth.theta_identity(L1, L2, D, 2, noise=1e-3, seed=seed)
    return p, lat, desc, th * scale


def _close_log(a, b, tol=1e-10):
    return np.all(np.abs(a - b) <= tol * np.maximum(1.0, np.abs(b)))


EVAL_CASES = [
    (3, 3, 2, 4, 0.0),     # exact chi
    (4, 4, 2, 4, 0.0),     # the small cooling lattice (exact chi)
    (4, 5, 3, 5, 0.0),     # truncating, ragged bond dimensions
    (4, 4, 2, 3, 0.5),     # J1-J2, truncating
    (8, 8, 4, 16, 0.0),    # the 8x8 throughput lattice
    (5, 5, 4, 24, 0.0),    # chi D = 96: general compression kernel, work matrices in the workspace
    (5, 5, 6, 12, 0.5),    # D = 6, J1-J2: general kernel, workspace-resident
]


@pytest.mark.parametrize("L1,L2,D,chi,J2", EVAL_CASES)
def test_eval_and_grad_match_oracle(L1, L2, D, chi, J2):
    dev = _dev()
    p, lat, desc, th = _setup(L1, L2, D, chi, J2)
    n = 3 if L1 * L2 >= 64 else 6
    cfg = synth.configs_sector(n, lat.N, 2, seed=L1 * 100 + chi)
    _say("eval", L1, L2, D, chi, J2, "n", n)
    theta_d = torch.tensor(th, device=dev)
    cfg_d = torch.tensor(cfg, device=dev)
    la, sg, el, st = p.peps_eval_batch(desc, theta_d, cfg_d)
    O, la2, st2 = p.peps_grad_batch(desc, theta_d, cfg_d)
    torch.cuda.synchronize()
    assert p.check(st) == 0 and p.check(st2) == 0
    ref = measure.evaluate_batch(lat, th, cfg, chi)
    la, sg, el, O, la2 = (x.cpu().numpy() for x in (la, sg, el, O, la2))
    assert _close_log(la, ref["log_abs"]), (la, ref["log_abs"])
    assert np.array_equal(la, la2)
    assert np.array_equal(sg, ref["sign"])
    emag = max(np.abs(ref["e_loc"]).mean(), 1e-300)
    assert np.all(np.abs(el - ref["e_loc"]) <= 1e-10 * np.maximum(np.abs(ref["e_loc"]), emag)), (el, ref["e_loc"])
    assert np.all(np.abs(O - ref["O"]) <= 1e-9 * np.maximum(1.0, np.abs(ref["O"])))


def _oracle_chains(lat, th, cfg, chi, seed, sweep0, n_sweeps, tie_tol=1e-12):
    out = []
    for ch in range(cfg.shape[0]):
        S = cfg[ch].astype(np.int64)
        acc = np.zeros(3, dtype=np.int64)
        ties = []
        meas = []
        for k in range(n_sweeps):
            res = sampler.sweep(lat, th, S, chi, seed, ch, sweep0 + k, tie_tol=tie_tol)
            S = res["S"]
            acc += res["n_accept"]
            ties += res["near_ties"]
            meas.append(measure.evaluate(lat, th, S, chi))
        out.append((S, acc, ties, meas))
    return out


SWEEP_CASES = [
    (4, 4, 2, 4, "identity", 4, 3),
    (4, 4, 2, 4, "random", 4, 2),
    (3, 4, 3, 6, "random", 4, 2),
    (4, 5, 3, 5, "random", 3, 2),
    (8, 8, 4, 16, "random", 2, 1),
    (5, 5, 4, 24, "random", 2, 1),
]


@pytest.mark.parametrize("L1,L2,D,chi,init,n_chains,n_sweeps", SWEEP_CASES)
def test_sample_sweep_bit_exact(L1, L2, D, chi, init, n_chains, n_sweeps):
    dev = _dev()
    p, lat, desc, th = _setup(L1, L2, D, chi, theta=init, seed=11)
    cfg = synth.configs_diagonal(n_chains, lat.N, 2, seed=5)
    seed, sweep0 = 20240905, 3
    _say("sweep", L1, L2, D, chi, init, n_chains, n_sweeps)
    theta_d = torch.tensor(th, device=dev)
    cfg_d = torch.tensor(cfg, device=dev)
    res = p.peps_sample_sweep(desc, theta_d, cfg_d, seed, sweep0, n_sweeps)
    torch.cuda.synchronize()
    assert p.check(res["status"]) == 0
    ref = _oracle_chains(lat, th, cfg, chi, seed, sweep0, n_sweeps)
    got_cfg = cfg_d.cpu().numpy()
    acc = res["n_accept"].cpu().numpy()
    e = res["e_loc"].cpu().numpy()
    la = res["log_abs"].cpu().numpy()
    O = res["O"].cpu().numpy()
    for ch, (S, a, ties, meas) in enumerate(ref):
        if ties:
            print("near-tie, chain", ch, ties)
            continue
        assert np.array_equal(got_cfg[ch], S.astype(np.uint8)), ch
        assert np.array_equal(acc[ch], a), (ch, acc[ch], a)
        for k in range(n_sweeps):
            m = meas[k]
            assert _close_log(la[k, ch], m["log_abs"])
            assert abs(e[k, ch] - m["e_loc"]) <= 1e-10 * max(abs(m["e_loc"]), 1.0)
            assert np.all(np.abs(O[k, ch] - m["O"]) <= 1e-9 * np.maximum(1.0, np.abs(m["O"])))


@pytest.mark.parametrize("L1,L2,D,chi", [(4, 4, 2, 4), (4, 5, 3, 5)])
def test_reweighted_sweep_bit_exact(L1, L2, D, chi):
    """alpha = 1 (Appendix A): acceptance on |R|, same bit-exact bar."""
    dev = _dev()
    import paper_2409_05285_amd as p
    lat = Lattice(L1, L2, D=D, chi=chi)
    desc = p.Desc(L1, L2, D, chi, alpha=1)
    th = synth.theta_identity(L1, L2, D, 2, noise=0.05, seed=13)
    cfg = synth.configs_diagonal(4, lat.N, 2, seed=14)
    seed, sweep0, n_sweeps = 77, 5, 2
    _say("reweighted sweep", L1, L2, D, chi)
    cfg_d = torch.tensor(cfg, device=dev)
    res = p.peps_sample_sweep(desc, torch.tensor(th, device=dev), cfg_d, seed, sweep0, n_sweeps)
    torch.cuda.synchronize()
    assert p.check(res["status"]) == 0
    got = cfg_d.cpu().numpy()
    acc = res["n_accept"].cpu().numpy()
    for ch in range(cfg.shape[0]):
        S = cfg[ch].astype(np.int64)
        a = np.zeros(3, dtype=np.int64)
        ties = []
        for k in range(n_sweeps):
            r = sampler.sweep(lat, th, S, chi, seed, ch, sweep0 + k, alpha=1)
            S, ties = r["S"], ties + r["near_ties"]
            a += r["n_accept"]
        if ties:
            continue
        assert np.array_equal(got[ch], S.astype(np.uint8)), ch
        assert np.array_equal(acc[ch], a), ch


@pytest.mark.parametrize("L1,L2,D,chi,mixed", [(4, 4, 2, 4, False), (8, 8, 4, 16, False), (8, 8, 4, 16, True),
                                               (4, 4, 6, 36, False)])
def test_identity_sweep_flips_every_site(L1, L2, D, chi, mixed):
    """At the exact beta = 0 state every site move (s, s) -> (1-s, 1-s) has
    ratio 1 and is accepted, and every bond move leads to s != s' (rho = 0)
    and is rejected: one sweep flips every site once."""
    dev = _dev()
    import paper_2409_05285_amd as p
    N = L1 * L2
    desc = p.Desc(L1, L2, D, chi, precision=p.PREC_MIXED if mixed else p.PREC_FP64)
    th = synth.theta_identity(L1, L2, D, 2)
    cfg = synth.configs_diagonal(8, N, 2, seed=9)
    _say(f"identity sweep {L1}x{L2} D={D} chi={chi} mixed={mixed}")
    cfg_d = torch.tensor(cfg, device=dev)
    res = p.peps_sample_sweep(desc, torch.tensor(th, device=dev), cfg_d, 1, 0, 1)
    torch.cuda.synchronize()
    assert p.check(res["status"]) == 0
    acc = res["n_accept"].cpu().numpy()
    assert np.all(acc[:, 0] == 0) and np.all(acc[:, 2] == 0) and np.all(acc[:, 1] == N)
    s = cfg // 2
    flipped = (1 - s) * 2 + (1 - s)
    assert np.array_equal(cfg_d.cpu().numpy(), flipped.astype(np.uint8))
    # beta = 0: log|psi| = 0
    assert np.allclose(res["log_abs"].cpu().numpy(), 0.0, atol=1e-4 if mixed else 1e-12)


def test_weighted_sr_cg_matches_oracle():
    dev = _dev()
    import paper_2409_05285_amd as p
    lat = Lattice(4, 4, D=2, chi=4)
    desc = p.Desc(4, 4, 2, 4)
    rng = np.random.default_rng(91)
    n_s = 120
    cfg = synth.configs_uniform(n_s, 16, 2, seed=92)
    O = rng.standard_normal((n_s, lat.nnz))
    e = rng.standard_normal(n_s)
    w = rng.uniform(0.05, 2.0, n_s)
    _say("weighted sr", n_s)
    dth, g, stats, st = p.sr_cg_solve(desc, torch.tensor(cfg, device=dev), torch.tensor(O, device=dev),
                                      torch.tensor(e, device=dev), 0.01, 1e-3, 40, 0.0,
                                      weights=torch.tensor(w, device=dev))
    torch.cuda.synchronize()
    # a fixed iteration count (rtol = 0) ends above the residual bar: warning, not error
    assert p.check(st) == 1 and stats[4].item() == 1.0
    ref = sr.sr_solve(lat, cfg, O, e, tau=0.01, eps=1e-3, max_iter=40, rtol=0.0, weights=w)
    dth, g, stats = dth.cpu().numpy(), g.cpu().numpy(), stats.cpu().numpy()
    assert np.allclose(g, ref["g"], rtol=1e-12, atol=1e-14 * np.abs(ref["g"]).max())
    assert np.all(np.abs(dth - ref["dtheta"]) <= 1e-9 * np.abs(ref["dtheta"]).max())
    assert abs(stats[0] - ref["ebar"]) <= 1e-13 * max(1.0, abs(ref["ebar"]))


@pytest.mark.parametrize("n_s,iters", [(40, 25), (300, 60)])
def test_sr_cg_matches_oracle(n_s, iters):
    dev = _dev()
    import paper_2409_05285_amd as p
    lat = Lattice(4, 4, D=2, chi=4)
    desc = p.Desc(4, 4, 2, 4)
    rng = np.random.default_rng(n_s)
    cfg = synth.configs_uniform(n_s, 16, 2, seed=n_s + 1)
    O = rng.standard_normal((n_s, lat.nnz))
    e = rng.standard_normal(n_s)
    _say("sr", n_s, iters)
    dth, g, stats, st = p.sr_cg_solve(desc, torch.tensor(cfg, device=dev), torch.tensor(O, device=dev),
                                      torch.tensor(e, device=dev), 0.01, 1e-3, iters, 0.0)
    torch.cuda.synchronize()
    # a fixed iteration count (rtol = 0) ends above the residual bar: warning, not error
    assert p.check(st) == 1 and stats[4].item() == 1.0
    ref = sr.sr_solve(lat, cfg, O, e, tau=0.01, eps=1e-3, max_iter=iters, rtol=0.0)
    dth, g, stats = dth.cpu().numpy(), g.cpu().numpy(), stats.cpu().numpy()
    assert np.allclose(g, ref["g"], rtol=1e-12, atol=1e-14 * np.abs(ref["g"]).max())
    scale = np.abs(ref["dtheta"]).max()
    assert np.all(np.abs(dth - ref["dtheta"]) <= 1e-9 * scale)
    assert stats[2] == ref["iters"]
    assert abs(stats[0] - ref["ebar"]) <= 1e-13
    # converged solve agrees with the dense solve
    dth2, _, stats2, st2 = p.sr_cg_solve(desc, torch.tensor(cfg, device=dev), torch.tensor(O, device=dev),
                                         torch.tensor(e, device=dev), 0.01, 1e-3, 2000, 1e-12)
    torch.cuda.synchronize()
    dense = sr.sr_solve_dense(lat, cfg, O, e, tau=0.01, eps=1e-3)
    assert np.allclose(dth2.cpu().numpy(), dense, rtol=1e-7, atol=1e-10 * np.abs(dense).max())
    assert stats2[2] < 2000
    assert p.check(st2) == 0 and stats2[4].item() == 0.0   # converged: no warning


# ---------------------------------------------------------------------------
# Mixed precision

MIXED_TOL = 1e-4

MIXED_EVAL_CASES = [
    (3, 3, 2, 4, 0.0, 1.0),
    (4, 5, 3, 5, 0.0, 1.0),
    (4, 4, 2, 3, 0.5, 1.0),
    (8, 8, 4, 16, 0.0, 1.0),
    (4, 8, 2, 4, 0.0, 1e-6),   # strip values far below the FP32 range without rescaling
    (4, 8, 2, 4, 0.0, 1e6),    # and far above it
]


@pytest.mark.parametrize("L1,L2,D,chi,J2,scale", MIXED_EVAL_CASES)
def test_mixed_eval_and_grad_match_oracle(L1, L2, D, chi, J2, scale):
    dev = _dev()
    p, lat, desc, th = _setup(L1, L2, D, chi, J2, mixed=True, scale=scale)
    n = 3 if L1 * L2 >= 64 else 6
    cfg = synth.configs_sector(n, lat.N, 2, seed=L1 * 100 + chi + 1)
    _say("mixed eval", L1, L2, D, chi, J2, scale, "n", n)
    theta_d = torch.tensor(th, device=dev)
    cfg_d = torch.tensor(cfg, device=dev)
    la, sg, el, st = p.peps_eval_batch(desc, theta_d, cfg_d)
    O, la2, st2 = p.peps_grad_batch(desc, theta_d, cfg_d)
    torch.cuda.synchronize()
    assert p.check(st) == 0 and p.check(st2) == 0
    ref = measure.evaluate_batch(lat, th, cfg, chi)
    la, sg, el, O, la2 = (x.cpu().numpy() for x in (la, sg, el, O, la2))
    assert _close_log(la, ref["log_abs"], MIXED_TOL), (la, ref["log_abs"])
    assert np.array_equal(la, la2)
    assert np.array_equal(sg, ref["sign"])
    emag = max(np.abs(ref["e_loc"]).mean(), 1e-300)
    err = np.abs(el - ref["e_loc"]) / np.maximum(np.abs(ref["e_loc"]), emag)
    print("mixed E_loc max rel err", err.max(), flush=True)
    assert np.all(err <= MIXED_TOL), (el, ref["e_loc"])
    omax = np.maximum(1.0, np.abs(ref["O"]).max(axis=1, keepdims=True))
    assert np.all(np.abs(O - ref["O"]) <= MIXED_TOL * omax)


MIXED_SWEEP_CASES = [
    (4, 4, 2, 4, "random", 6, 2),
    (4, 5, 3, 5, "random", 4, 2),
    (8, 8, 4, 16, "random", 2, 1),
]


@pytest.mark.parametrize("L1,L2,D,chi,init,n_chains,n_sweeps", MIXED_SWEEP_CASES)
def test_mixed_sample_sweep(L1, L2, D, chi, init, n_chains, n_sweeps):
    dev = _dev()
    p, lat, desc, th = _setup(L1, L2, D, chi, theta=init, seed=11, mixed=True)
    cfg = synth.configs_diagonal(n_chains, lat.N, 2, seed=5)
    seed, sweep0 = 20240905, 3
    _say("mixed sweep", L1, L2, D, chi, init, n_chains, n_sweeps)
    theta_d = torch.tensor(th, device=dev)
    cfg_d = torch.tensor(cfg, device=dev)
    res = p.peps_sample_sweep(desc, theta_d, cfg_d, seed, sweep0, n_sweeps)
    torch.cuda.synchronize()
    assert p.check(res["status"]) == 0
    ref = _oracle_chains(lat, th, cfg, chi, seed, sweep0, n_sweeps, tie_tol=MIXED_TOL)
    got_cfg = cfg_d.cpu().numpy()
    acc = res["n_accept"].cpu().numpy()
    e = res["e_loc"].cpu().numpy()
    la = res["log_abs"].cpu().numpy()
    compared = 0
    for ch, (S, a, ties, meas) in enumerate(ref):
        if ties:
            print("near-tie, chain", ch, ties)
            continue
        compared += 1
        assert np.array_equal(got_cfg[ch], S.astype(np.uint8)), ch
        assert np.array_equal(acc[ch], a), (ch, acc[ch], a)
        for k in range(n_sweeps):
            m = meas[k]
            assert _close_log(la[k, ch], m["log_abs"], MIXED_TOL)
            assert abs(e[k, ch] - m["e_loc"]) <= MIXED_TOL * max(abs(m["e_loc"]), 1.0)
    assert compared >= 1


# ---------------------------------------------------------------------------
# Fermi-Hubbard (d = 4): hops with Jordan-Wigner signs, plain tensors


def _hub_setup(L1, L2, D, chi, mixed=False, seed=21):
    import paper_2409_05285_amd as p
    from oracle.lattice import MODEL_HUBBARD
    lat = Lattice(L1, L2, D=D, chi=chi, d=4, model=MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0)
    desc = p.Desc(L1, L2, D, chi, d=4, model=p.MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0,
                  precision=p.PREC_MIXED if mixed else p.PREC_FP64)
    th = synth.theta_random_unit(L1, L2, D, 4, seed=seed)
    return p, lat, desc, th


@pytest.mark.parametrize("L1,L2,D,chi,mixed", [(3, 3, 2, 4, False), (4, 4, 2, 4, False), (3, 4, 2, 3, False),
                                               (4, 4, 2, 4, True),
                                               # chi D = 80: the workspace-resident compression kernel
                                               (4, 4, 4, 20, False), (5, 5, 4, 20, False), (5, 5, 4, 20, True)])
def test_hubbard_eval_and_grad_match_oracle(L1, L2, D, chi, mixed):
    dev = _dev()
    p, lat, desc, th = _hub_setup(L1, L2, D, chi, mixed)
    cfg = synth.configs_sector(5, lat.N, 4, seed=L1 * 10 + L2)
    _say("hubbard eval", L1, L2, D, chi, mixed)
    theta_d = torch.tensor(th, device=dev)
    cfg_d = torch.tensor(cfg, device=dev)
    la, sg, el, st = p.peps_eval_batch(desc, theta_d, cfg_d)
    O, la2, st2 = p.peps_grad_batch(desc, theta_d, cfg_d)
    torch.cuda.synchronize()
    assert p.check(st) == 0 and p.check(st2) == 0
    ref = measure.evaluate_batch(lat, th, cfg, chi)
    la, sg, el, O = (x.cpu().numpy() for x in (la, sg, el, O))
    tol = MIXED_TOL if mixed else 1e-10
    assert _close_log(la, ref["log_abs"], tol), (la, ref["log_abs"])
    assert np.array_equal(sg, ref["sign"])
    emag = max(np.abs(ref["e_loc"]).mean(), 1e-300)
    assert np.all(np.abs(el - ref["e_loc"]) <= tol * np.maximum(np.abs(ref["e_loc"]), emag)), (el, ref["e_loc"])
    otol = MIXED_TOL * np.maximum(1.0, np.abs(ref["O"]).max(axis=1, keepdims=True)) if mixed else \
        1e-9 * np.maximum(1.0, np.abs(ref["O"]))
    assert np.all(np.abs(O - ref["O"]) <= otol)


def test_hubbard_sweep_bit_exact():
    dev = _dev()
    p, lat, desc, th = _hub_setup(4, 4, 2, 4)
    cfg = synth.configs_diagonal(3, lat.N, 4, seed=23)
    seed, sweep0, n_sweeps = 99, 1, 2
    _say("hubbard sweep")
    cfg_d = torch.tensor(cfg, device=dev)
    res = p.peps_sample_sweep(desc, torch.tensor(th, device=dev), cfg_d, seed, sweep0, n_sweeps)
    torch.cuda.synchronize()
    assert p.check(res["status"]) == 0
    ref = _oracle_chains(lat, th, cfg, 4, seed, sweep0, n_sweeps)
    got = cfg_d.cpu().numpy()
    acc = res["n_accept"].cpu().numpy()
    e = res["e_loc"].cpu().numpy()
    compared = 0
    for ch, (S, a, ties, meas) in enumerate(ref):
        if ties:
            continue
        compared += 1
        assert np.array_equal(got[ch], S.astype(np.uint8)), ch
        assert np.array_equal(acc[ch], a), (ch, acc[ch], a)
        m = meas[-1]
        assert abs(e[-1, ch] - m["e_loc"]) <= 1e-10 * max(abs(m["e_loc"]), 1.0)
    assert compared >= 1


@pytest.mark.parametrize("mixed", [False, True])
def test_multi_sweep_call_matches_single_sweeps(mixed):
    """One call of n sweeps (bottom boundaries of each measurement reused by
    the next sweep) against n calls of one sweep (recomputed each call):
    bit-identical configurations, per-sweep sample configurations,
    measurements and accept counts."""
    dev = _dev()
    p, lat, desc, th = _setup(4, 5, 3, 5, theta="random", seed=41, mixed=mixed)
    cfg = synth.configs_diagonal(6, lat.N, 2, seed=42)
    seed, sweep0, ns = 9090, 11, 3
    _say("multi-sweep call", "mixed" if mixed else "fp64")
    theta_d = torch.tensor(th, device=dev)
    cfg_a = torch.tensor(cfg, device=dev)
    ra = p.peps_sample_sweep(desc, theta_d, cfg_a, seed, sweep0, ns, want_configs=True)
    cfg_b = torch.tensor(cfg, device=dev)
    acc_b = torch.zeros((cfg.shape[0], 3), dtype=torch.int32, device=dev)
    rb = []
    for k in range(ns):
        r = p.peps_sample_sweep(desc, theta_d, cfg_b, seed, sweep0 + k, 1, n_accept=acc_b, want_configs=True)
        rb.append({key: r[key].clone() for key in ("log_abs", "e_loc", "O", "configs")})
    torch.cuda.synchronize()
    assert p.check(ra["status"]) == 0
    assert torch.equal(cfg_a, cfg_b)
    assert torch.equal(ra["n_accept"], acc_b)
    for k in range(ns):
        for key in ("log_abs", "e_loc", "O", "configs"):
            assert torch.equal(ra[key][k], rb[k][key][0]), (k, key)
    assert torch.equal(ra["configs"][ns - 1], cfg_a)


def test_parity_even_hubbard_ansatz():
    """Z2-graded (parity-even) Hubbard tensors: even configurations match the
    oracle at the usual bars, a sweep from the diagonal start is bit-exact
    and stays in the even sector, and configurations of odd total parity
    have zero amplitude (reported through the status word, log|psi| = -inf)."""
    dev = _dev()
    import paper_2409_05285_amd as p
    from oracle.lattice import MODEL_HUBBARD
    L1, L2, D, chi = 3, 4, 2, 4
    lat = Lattice(L1, L2, D=D, chi=chi, d=4, model=MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0)
    desc = p.Desc(L1, L2, D, chi, d=4, model=p.MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0)
    th = synth.theta_random_parity_even(L1, L2, D, 4, seed=91)
    theta_d = torch.tensor(th, device=dev)
    _say("parity-even hubbard")
    # even sector: sector-consistent configurations have even total parity
    cfg = synth.configs_sector(4, lat.N, 4, seed=92)
    assert all(sum(bin(int(x)).count("1") for x in S) % 2 == 0 for S in cfg)
    la, sg, el, st = p.peps_eval_batch(desc, theta_d, torch.tensor(cfg, device=dev))
    torch.cuda.synchronize()
    assert p.check(st) == 0
    ref = measure.evaluate_batch(lat, th, cfg, chi, want_O=False)
    la, sg, el = (x.cpu().numpy() for x in (la, sg, el))
    assert _close_log(la, ref["log_abs"])
    assert np.array_equal(sg, ref["sign"])
    emag = max(np.abs(ref["e_loc"]).mean(), 1e-300)
    assert np.all(np.abs(el - ref["e_loc"]) <= 1e-10 * np.maximum(np.abs(ref["e_loc"]), emag))
    # one sweep from the diagonal start: bit-exact, even parity kept
    cfg0 = synth.configs_diagonal(3, lat.N, 4, seed=93)
    cfg_d = torch.tensor(cfg0, device=dev)
    res = p.peps_sample_sweep(desc, theta_d, cfg_d, 4321, 2, 1)
    torch.cuda.synchronize()
    assert p.check(res["status"]) == 0
    got = cfg_d.cpu().numpy()
    for ch in range(cfg0.shape[0]):
        r = sampler.sweep(lat, th, cfg0[ch].astype(np.int64), chi, 4321, ch, 2)
        if r["near_ties"]:
            continue
        assert np.array_equal(got[ch], r["S"].astype(np.uint8)), ch
        assert sum(bin(int(x)).count("1") for x in got[ch]) % 2 == 0
    # odd total parity: zero amplitude, reported through the status word.
    # The QR sweep's reflectors may mix the parity sectors of a bond (a valid
    # gauge), so the device's amplitude is zero only to rounding: at least
    # 1e-13 below the even configurations' amplitudes.
    odd = cfg[:2].copy()
    odd[:, 0] = odd[:, 0] ^ 1          # flip the bra up-occupation of site 0
    la_o, _, _, st_o = p.peps_eval_batch(desc, theta_d, torch.tensor(odd, device=dev))
    torch.cuda.synchronize()
    assert int(st_o.item()) in (-6, -5)
    la_o = la_o.cpu().numpy()
    assert np.all(np.isneginf(la_o) | (la_o < la.min() + math.log(1e-13))), (la_o, la)
    # declared Z2-graded tensors (fermionic = 1): the odd configurations have
    # amplitude exactly 0, decided from the digits (bit-exact: -inf, sign 0,
    # status -6), and the even ones are unchanged bit for bit
    descf = p.Desc(L1, L2, D, chi, d=4, model=p.MODEL_HUBBARD, t=1.0, U=8.0, mu=4.0, fermionic=1)
    la_f, sg_f, _, st_f = p.peps_eval_batch(descf, theta_d, torch.tensor(odd, device=dev))
    torch.cuda.synchronize()
    assert int(st_f.item()) == -6
    assert np.all(np.isneginf(la_f.cpu().numpy())) and np.all(sg_f.cpu().numpy() == 0)
    la_e, sg_e, el_e, st_e = p.peps_eval_batch(descf, theta_d, torch.tensor(cfg, device=dev))
    torch.cuda.synchronize()
    assert p.check(st_e) == 0
    assert np.array_equal(la_e.cpu().numpy(), la) and np.array_equal(sg_e.cpu().numpy(), sg)
    assert np.array_equal(el_e.cpu().numpy(), el)
    # a chain started in the odd sector cannot move: reported, configuration kept
    cfg_o = torch.tensor(odd, device=dev)
    res_o = p.peps_sample_sweep(descf, theta_d, cfg_o, 4321, 2, 1, measure=False)
    torch.cuda.synchronize()
    assert int(res_o["status"].item()) == -6
    assert np.array_equal(cfg_o.cpu().numpy(), odd)


def test_out_of_range_digit_is_reported_not_read():
    """A configuration digit >= d^2 given straight to the C ABI (past the
    binding's own check): every kernel reads it as 0, nothing outside theta
    or the parameter vectors is touched, and the status word records
    PEPS_ERR_ARG (-1); evaluation, a sweep and the SR solve."""
    dev = _dev()
    import ctypes

    import paper_2409_05285_amd as p
    from paper_2409_05285_amd import api
    from paper_2409_05285_amd._lib import LIB
    _say("out-of-range digit")
    desc = p.Desc(4, 4, 2, 4)
    th = torch.tensor(synth.theta_random_unit(4, 4, 2, 2, seed=3), device=dev)
    cfg = synth.configs_diagonal(4, 16, 2, seed=4)
    cfg[2, 5] = 200                                   # far past d^2 = 4
    cfg_d = torch.tensor(cfg, device=dev)
    n = 4
    la = torch.empty(n, dtype=torch.float64, device=dev)
    sg = torch.empty(n, dtype=torch.int8, device=dev)
    el = torch.empty(n, dtype=torch.float64, device=dev)
    st = p.new_status(dev)
    ws = torch.empty(p.workspace_bytes(desc, n, "eval"), dtype=torch.uint8, device=dev)
    c = desc.c()
    code = LIB.peps_eval_batch(ctypes.byref(c), api._ptr(th), n, api._ptr(cfg_d), api._ptr(la), api._ptr(sg),
                               api._ptr(el), api._ptr(st), api._ptr(ws), ws.numel(), None, api._stream())
    torch.cuda.synchronize()
    assert code == 0 and int(st.item()) == -1
    # the binding refuses the same input before any launch
    with pytest.raises(ValueError):
        p.peps_eval_batch(desc, th, cfg_d)
    # a sweep and the SR solve through the ABI
    st2 = p.new_status(dev)
    ws2 = torch.empty(p.workspace_bytes(desc, n, "sweep"), dtype=torch.uint8, device=dev)
    code = LIB.peps_sample_sweep(ctypes.byref(c), api._ptr(th), n, api._ptr(cfg_d), 1, 0, None, 1, None, None,
                                 None, None, None, None, api._ptr(st2), api._ptr(ws2), ws2.numel(), None,
                                 api._stream())
    torch.cuda.synchronize()
    assert code == 0 and int(st2.item()) == -1
    nnz = p.peps_orow_count(desc)
    O = torch.zeros((n, nnz), dtype=torch.float64, device=dev)
    e = torch.zeros(n, dtype=torch.float64, device=dev)
    dth = torch.empty(p.peps_param_count(desc), dtype=torch.float64, device=dev)
    stats = torch.zeros(5, dtype=torch.float64, device=dev)
    st3 = p.new_status(dev)
    bad = torch.tensor(cfg, device=dev)
    ws3 = torch.empty(p.workspace_bytes(desc, n, "sr"), dtype=torch.uint8, device=dev)
    code = LIB.sr_cg_solve(ctypes.byref(c), n, api._ptr(bad), api._ptr(O), None, None, api._ptr(e), 0.01, 1e-3, 5,
                           0.0, api._ptr(dth), None, None, api._ptr(stats), api._ptr(st3), api._ptr(ws3),
                           ws3.numel(), None, api._stream())
    torch.cuda.synchronize()
    assert code == 0 and int(st3.item()) == -1
