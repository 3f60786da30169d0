"""Parity at the large bond dimension of the 12x12 J1-J2 workload (J2/J1 =
0.5, open boundaries, d^2 = 4, D = 6, chi = 36, so chi D = 216): the
boundary compression runs in the workspace-resident kernel (blocked
Householder QR with compact WY updates, Jacobi SVD in the workspace).

Samples: random unit-Frobenius tensors (seed 103), two sector-consistent
configurations for evaluation and gradients, and one chain for a sweep,
each recomputed by the oracle from the same seeded inputs.

Bars.  Configurations, accept counts and signs bit-exact; mixed precision
1e-4 as elsewhere; FP64 the bars of every other lattice: log|psi| and
E_loc 1e-10, O 1e-9.  At this depth (eleven truncations of 216 to 36 per
boundary) these quantities are conditioned near those bars: the oracle run
with LAPACK's gesvd instead of gesdd for the same SVDs (both exact to
rounding) moves O by up to 7e-10 on these samples, and the eval test
recomputes and prints that spread for its first sample.  The device's
Jacobi therefore refines its rotation angle to full precision and stops one
quadratic step later than the small-shape kernel.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import measure, sampler
from oracle.lattice import Lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

L1 = L2 = 12
D, CHI, J2 = 6, 36, 0.5


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _driver_spread(lat, th, S):
    """The oracle's own disagreement between two exact SVD drivers (LAPACK
    gesdd, numpy's default, and gesvd) on one sample."""
    import scipy.linalg
    a = measure.evaluate(lat, th, S, CHI)
    orig = np.linalg.svd
    np.linalg.svd = lambda x, full_matrices=False: scipy.linalg.svd(x, full_matrices=full_matrices,
                                                                    lapack_driver="gesvd")
    try:
        b = measure.evaluate(lat, th, S, CHI)
    finally:
        np.linalg.svd = orig
    return (abs(a["log_abs"] - b["log_abs"]), abs(a["e_loc"] - b["e_loc"]) / max(1.0, abs(a["e_loc"])),
            float((np.abs(a["O"] - b["O"]) / np.maximum(1.0, np.abs(a["O"]))).max()))


@pytest.mark.parametrize("mixed", [False, True])
def test_large_chi_eval_and_grad(mixed):
    dev = _dev()
    import paper_2409_05285_amd as p
    _say("12x12 J1-J2 D=6 chi=36 eval", "mixed" if mixed else "fp64")
    lat = Lattice(L1, L2, D=D, chi=CHI, J1=1.0, J2=J2)
    desc = p.Desc(L1, L2, D, CHI, J1=1.0, J2=J2, precision=p.PREC_MIXED if mixed else p.PREC_FP64)
    th = synth.theta_random_unit(L1, L2, D, 2, seed=103)
    cfg = synth.configs_sector(2, lat.N, 2, seed=1203)
    theta_d = torch.tensor(th, device=dev)
    cfg_d = torch.tensor(cfg, device=dev)
    import time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    la, sg, el, st = p.peps_eval_batch(desc, theta_d, cfg_d)
    O, la2, st2 = p.peps_grad_batch(desc, theta_d, cfg_d)
    torch.cuda.synchronize()
    print("[time] device eval + grad of %d samples: %.2f s" % (cfg.shape[0], time.perf_counter() - t0), flush=True)
    assert p.check(st) == 0 and p.check(st2) == 0
    ref = measure.evaluate_batch(lat, th, cfg, CHI)
    la, sg, el, O = (x.cpu().numpy() for x in (la, sg, el, O))
    if not mixed:
        spread = _driver_spread(lat, th, cfg[0])
        print("[oracle] gesdd vs gesvd on sample 0: log|psi| %.2e, E_loc rel %.2e, O rel %.2e" % spread, flush=True)
    tol = 1e-4 if mixed else 1e-10
    emag0 = max(np.abs(ref["e_loc"]).mean(), 1e-300)
    print("[err] log|psi| %.2e  E_loc %.2e  O %.2e" % (
        (np.abs(la - ref["log_abs"]) / np.maximum(1.0, np.abs(ref["log_abs"]))).max(),
        (np.abs(el - ref["e_loc"]) / np.maximum(np.abs(ref["e_loc"]), emag0)).max(),
        (np.abs(O - ref["O"]) / np.maximum(1.0, np.abs(ref["O"]))).max()), flush=True)
    assert np.all(np.abs(la - ref["log_abs"]) <= tol * np.maximum(1.0, np.abs(ref["log_abs"]))), (la, ref["log_abs"])
    assert np.array_equal(sg, ref["sign"])
    emag = max(np.abs(ref["e_loc"]).mean(), 1e-300)
    assert np.all(np.abs(el - ref["e_loc"]) <= tol * np.maximum(np.abs(ref["e_loc"]), emag)), (el, ref["e_loc"])
    if mixed:
        for i in range(O.shape[0]):
            assert np.all(np.abs(O[i] - ref["O"][i]) <= 1e-4 * np.abs(ref["O"][i]).max())
    else:
        rel = np.abs(O - ref["O"]) / np.maximum(1.0, np.abs(ref["O"]))
        worst = np.argsort(rel.ravel())[-5:]
        print("[O] worst relative errors", rel.ravel()[worst], "values", ref["O"].ravel()[worst],
              "entries", worst % O.shape[1], flush=True)
        assert np.all(rel <= 1e-9)


def test_large_chi_sweep_bit_exact():
    dev = _dev()
    import paper_2409_05285_amd as p
    _say("12x12 J1-J2 D=6 chi=36 sweep")
    lat = Lattice(L1, L2, D=D, chi=CHI, J1=1.0, J2=J2)
    desc = p.Desc(L1, L2, D, CHI, J1=1.0, J2=J2)
    th = synth.theta_random_unit(L1, L2, D, 2, seed=103)
    cfg = synth.configs_diagonal(1, lat.N, 2, seed=1204)
    seed = 777
    cfg_d = torch.tensor(cfg, device=dev)
    res = p.peps_sample_sweep(desc, torch.tensor(th, device=dev), cfg_d, seed, 0, 1)
    torch.cuda.synchronize()
    assert p.check(res["status"]) == 0
    r = sampler.sweep(lat, th, cfg[0].astype(np.int64), CHI, seed, 0, 0, tie_tol=1e-12)
    if r["near_ties"]:
        pytest.skip("near-tie in the oracle's Metropolis tests: %r" % (r["near_ties"],))
    assert np.array_equal(cfg_d.cpu().numpy()[0], r["S"].astype(np.uint8))
    assert np.array_equal(res["n_accept"].cpu().numpy()[0], r["n_accept"])
    m = measure.evaluate(lat, th, r["S"], CHI)
    la = float(res["log_abs"].cpu().numpy()[0, 0])
    e = float(res["e_loc"].cpu().numpy()[0, 0])
    assert abs(la - m["log_abs"]) <= 1e-10 * max(1.0, abs(m["log_abs"]))
    assert abs(e - m["e_loc"]) <= 1e-10 * max(abs(m["e_loc"]), 1.0)


def test_large_chi_last_row_O_matches_central_differences():
    """The adjoint O rows against central differences of log|psi| (h = 1e-6,
    FP64) at this lattice's full shape.  For an entry of the last row the
    identity is exact under truncation: log|psi| = log|rho_{L1-1}|, the top
    boundary above that row does not depend on it and rho_{L1-1} is linear in
    it, so d log|psi| / d theta_k = O_k; a sample whose slice at that site
    differs has derivative 0.  Six entries (largest |O| of a site block, three
    per sample), both samples evaluated at every shift."""
    dev = _dev()
    import paper_2409_05285_amd as p
    _say("12x12 J1-J2 D=6 chi=36 O vs central differences")
    lat = Lattice(L1, L2, D=D, chi=CHI, J1=1.0, J2=J2)
    desc = p.Desc(L1, L2, D, CHI, J1=1.0, J2=J2)
    th = synth.theta_random_unit(L1, L2, D, 2, seed=103)
    cfg = synth.configs_sector(2, lat.N, 2, seed=1203)
    cfg_d = torch.tensor(cfg, device=dev)
    theta_d = torch.tensor(th, device=dev)
    O, la0, st = p.peps_grad_batch(desc, theta_d, cfg_d)
    torch.cuda.synchronize()
    assert p.check(st) == 0
    O = O.cpu().numpy()
    poff, _ = lat.param_offsets()
    ooff, _ = lat.orow_offsets()
    r = L1 - 1
    picks = []
    for j, cols in ((0, (1, 5, 10)), (1, (0, 6, 11))):
        for c in cols:
            i = lat.site(r, c)
            bs = lat.block_size(r, c)
            q = int(np.argmax(np.abs(O[j, ooff[i]:ooff[i] + bs])))
            picks.append((i, int(cfg[j, i]), bs, q))
    h = 1e-6
    for (i, s, bs, q) in picks:
        k = poff[i] + s * bs + q
        vals = []
        for sgn in (1.0, -1.0):
            t = th.copy()
            t[k] += sgn * h
            la, _, _, st = p.peps_eval_batch(desc, torch.tensor(t, device=dev), cfg_d)
            torch.cuda.synchronize()
            assert p.check(st) == 0
            vals.append(la.cpu().numpy())
        fd = (vals[0] - vals[1]) / (2 * h)
        for j in range(2):
            want = O[j, ooff[i] + q] if int(cfg[j, i]) == s else 0.0
            print("[fd] site %d slice %d entry %d sample %d: O %.12f fd %.12f" % (i, s, q, j, want, fd[j]), flush=True)
            assert abs(fd[j] - want) <= 1e-5 * max(1.0, abs(want)), (i, q, j, fd[j], want)
