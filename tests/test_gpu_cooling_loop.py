"""The cooling loop (paper_2409_05285_amd.cool): one JSON record per SR
step with the documented fields; its steps equal the same library calls
made directly, bit for bit; a run resumed from (theta, configs, gsweep,
step) equals the uninterrupted run; the reweighted (alpha = 1) path runs."""
import io
import json
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = {"step", "beta_phys", "alpha", "E_per_site", "E_stderr", "accepted_per_sweep", "cg_iters",
        "cg_rel_residual", "cg_converged", "dtheta_norm", "samples_per_s", "gsweep"}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def _state(dev):
    th = torch.tensor(synth.theta_identity(4, 4, 2, 2, noise=1e-2, seed=21), device=dev)
    cfg = torch.tensor(synth.configs_diagonal(32, 16, 2, seed=22), device=dev)
    return th, cfg


def test_cooling_loop_records_and_direct_calls():
    dev = _dev()
    import paper_2409_05285_amd as p
    print("[case] cooling loop", flush=True)
    sys.stdout.flush()
    desc = p.Desc(4, 4, 2, 4)
    seed, S, tau, eps = 99, 3, 0.02, 1e-4
    th_a, cfg_a = _state(dev)
    buf = io.StringIO()
    recs = p.cool(desc, th_a, cfg_a, 2, S, tau, eps, seed, cg_iters=40, log=buf)
    lines = [json.loads(x) for x in buf.getvalue().splitlines()]
    assert len(lines) == 2 and all(set(x) == KEYS for x in lines)
    assert [x["beta_phys"] for x in lines] == [0.0, 4 * tau]
    assert lines[-1]["gsweep"] == 2 * S and recs[-1]["gsweep"] == 2 * S
    assert all(np.isfinite(x["E_per_site"]) and x["cg_iters"] > 0 for x in lines)
    # the same steps through the calls themselves
    th_b, cfg_b = _state(dev)
    nnz = p.peps_orow_count(desc)
    for k in range(2):
        res = p.peps_sample_sweep(desc, th_b, cfg_b, seed, k * S, S, want_configs=True)
        p.sr_cg_solve(desc, res["configs"].view(S * 32, 16), res["O"].view(S * 32, nnz), res["e_loc"].view(S * 32),
                      tau, eps, 40, 1e-10, want_g=False, theta=th_b)
    torch.cuda.synchronize()
    assert torch.equal(th_a, th_b) and torch.equal(cfg_a, cfg_b)
    # resumed run
    th_c, cfg_c = _state(dev)
    r1 = p.cool(desc, th_c, cfg_c, 1, S, tau, eps, seed, cg_iters=40)
    saved = (th_c.cpu().numpy(), cfg_c.cpu().numpy(), r1[-1]["gsweep"])
    th_d = torch.tensor(saved[0], device=dev)
    cfg_d = torch.tensor(saved[1], device=dev)
    r2 = p.cool(desc, th_d, cfg_d, 1, S, tau, eps, seed, cg_iters=40, step0=1, gsweep0=saved[2])
    assert torch.equal(th_a, th_d) and torch.equal(cfg_a, cfg_d)
    assert r2[0]["E_per_site"] == recs[1]["E_per_site"] and r2[0]["beta_phys"] == recs[1]["beta_phys"]


def test_cooling_loop_reweighted_sampling():
    dev = _dev()
    import paper_2409_05285_amd as p
    print("[case] cooling loop alpha = 1", flush=True)
    desc = p.Desc(4, 4, 2, 4, alpha=1)
    th, cfg = _state(dev)
    recs = p.cool(desc, th, cfg, 2, 2, 0.02, 1e-4, 5, cg_iters=40)
    assert len(recs) == 2 and all(np.isfinite(r["E_per_site"]) and np.isfinite(r["dtheta_norm"]) for r in recs)
    assert all(r["alpha"] == 1 for r in recs)


def test_cooling_loop_alpha_switch_and_device_weights():
    """alpha = 1 up to beta_phys = 0.3, then alpha = 2 (Benchmark section,
    Heisenberg paragraph: reweighted sampling until beta ~ 0.3).  The loop's
    steps equal direct calls bit for bit (sr_cg_solve with the log-amplitudes,
    so the library forms the Eq. A1 weights |rho| on the device); the logged
    energy equals the |rho|-weighted mean formed on the host; and the device
    weights give the same gradient as host weights exp(log|psi| - max)
    passed explicitly (to the rounding of exp)."""
    dev = _dev()
    import paper_2409_05285_amd as p
    print("[case] cooling loop alpha switch", flush=True)
    desc = p.Desc(4, 4, 2, 4, alpha=1)
    seed, S, tau, eps, steps = 17, 2, 0.05, 1e-4, 4
    th_a, cfg_a = _state(dev)
    recs = p.cool(desc, th_a, cfg_a, steps, S, tau, eps, seed, cg_iters=30, alpha_switch_beta=0.3)
    assert [r["alpha"] for r in recs] == [1, 1, 2, 2]        # beta_phys 0, 0.2, 0.4, 0.6
    th_b, cfg_b = _state(dev)
    nnz = p.peps_orow_count(desc)
    d2 = p.Desc(4, 4, 2, 4, alpha=2)
    for k in range(steps):
        d = desc if 4 * tau * k < 0.3 else d2
        res = p.peps_sample_sweep(d, th_b, cfg_b, seed, k * S, S, want_configs=True)
        la = res["log_abs"].view(S * 32)
        cf, O, e = res["configs"].view(S * 32, 16), res["O"].view(S * 32, nnz), res["e_loc"].view(S * 32)
        la_h = la.cpu().numpy()
        w_h = np.exp(la_h - la_h.max()) if d.alpha == 1 else np.ones_like(la_h)
        if d.alpha == 1:
            _, g_dev, _, _ = p.sr_cg_solve(d, cf, O, e, tau, eps, 0, 0.0, log_abs=la)
            _, g_host, _, _ = p.sr_cg_solve(d, cf, O, e, tau, eps, 0, 0.0, weights=torch.tensor(w_h, device=dev))
            gd, gh = g_dev.cpu().numpy(), g_host.cpu().numpy()
            assert np.allclose(gd, gh, rtol=0, atol=1e-12 * np.abs(gh).max())
        p.sr_cg_solve(d, cf, O, e, tau, eps, 30, 1e-10, log_abs=la, want_g=False, theta=th_b)
        eh = e.cpu().numpy()
        E = float((w_h * eh).sum() / w_h.sum()) / 32.0
        assert abs(recs[k]["E_per_site"] - E) <= 1e-12 * max(1.0, abs(E)), (k, recs[k]["E_per_site"], E)
    torch.cuda.synchronize()
    assert torch.equal(cfg_a, cfg_b)
    assert torch.equal(th_a, th_b)
