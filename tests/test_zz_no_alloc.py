"""sr_cg_solve_noalloc (no workspace argument; the library's fixed per-GPU
scratch) against sr_cg_solve with a caller workspace, through the C ABI:
two calls in a row, the second on a smaller input, with the plain and the
|rho|-weighted averages.  Both run the same kernels with the same layout, so
the results (dtheta, g, stats, the updated theta) are compared bit for
bit."""
import ctypes
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def _inputs(p, desc, n_s, seed, dev):
    rng = np.random.default_rng(seed)
    nnz = p.peps_orow_count(desc)
    cfg = torch.tensor(synth.configs_uniform(n_s, desc.N, 2, seed=seed + 1), device=dev)
    O = torch.tensor(rng.standard_normal((n_s, nnz)), device=dev)
    e = torch.tensor(rng.standard_normal(n_s) * 3.0 - 1.0, device=dev)
    la = torch.tensor(rng.standard_normal(n_s), device=dev)
    theta = torch.tensor(synth.theta_random_unit(desc.L1, desc.L2, desc.D, 2, seed=seed + 2), device=dev)
    return cfg, O, e, la, theta


def test_noalloc_solve_matches_workspace_solve():
    dev = _dev()
    import paper_2409_05285_amd as p
    from paper_2409_05285_amd import api
    from paper_2409_05285_amd._lib import LIB
    desc = p.Desc(8, 8, 4, 16, alpha=1)
    for call, (n_s, use_la) in enumerate(((3000, False), (700, True))):
        print("[case] noalloc call", call, "n_s", n_s, "log_abs weights" if use_la else "uniform", flush=True)
        sys.stdout.flush()
        cfg, O, e, la, theta = _inputs(p, desc, n_s, 50 + call, dev)
        lw = la if use_la else None
        th_ref = theta.clone()
        dth_ref, g_ref, st_ref, s_ref = p.sr_cg_solve(desc, cfg, O, e, 0.02, 1e-3, 60, 1e-12, log_abs=lw,
                                                      theta=th_ref)
        n_p = p.peps_param_count(desc)
        th = theta.clone()
        dth = torch.empty(n_p, dtype=torch.float64, device=dev)
        g = torch.empty(n_p, dtype=torch.float64, device=dev)
        stats = torch.zeros(5, dtype=torch.float64, device=dev)
        status = p.new_status(dev)
        c = desc.c()
        code = LIB.sr_cg_solve_noalloc(ctypes.byref(c), n_s, api._ptr(cfg), api._ptr(O), None, api._ptr(lw),
                                       api._ptr(e), 0.02, 1e-3, 60, 1e-12, api._ptr(dth), api._ptr(g), api._ptr(th),
                                       api._ptr(stats), api._ptr(status), api._stream())
        torch.cuda.synchronize()
        assert code == 0
        assert p.check(status) in (0, 1) and p.check(s_ref) in (0, 1)
        assert int(status.item()) == int(s_ref.item())
        assert torch.equal(dth, dth_ref)
        assert torch.equal(g, g_ref)
        assert torch.equal(stats, st_ref)
        assert torch.equal(th, th_ref)
        assert not torch.equal(th, theta)
    # the binding of the same entry point, with caller-owned outputs
    out = {"dtheta": torch.empty(p.peps_param_count(desc), dtype=torch.float64, device=dev), "g": None,
           "stats": torch.zeros(5, dtype=torch.float64, device=dev)}
    dth2, g2, st2, _ = p.sr_cg_solve_noalloc(desc, cfg, O, e, 0.02, 1e-3, 60, 1e-12, log_abs=la, out=out)
    torch.cuda.synchronize()
    assert g2 is None and torch.equal(dth2, dth_ref) and dth2 is out["dtheta"]
