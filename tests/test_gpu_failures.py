"""Data-dependent failures reported through the device status word, and
resuming from a saved state.

* A non-finite entry in theta: evaluation reports PEPS_ERR_NONFINITE (-5).
* A sample whose amplitude is exactly zero (the beta = 0 identity state and
  a configuration with s != s' at a site): evaluation and a sweep report
  PEPS_ERR_ZERO_AMPLITUDE (-6), the first error recorded, and log|psi| is
  -inf.
* Resume: two SR steps (sweeps with measurement, CG solve, update in place)
  against one step, a save of (theta, configs, next global sweep) to .npz,
  a reload into fresh device tensors and one more step: bit-identical theta
  and configurations (the Metropolis uniforms are positional, every
  reduction has a fixed order).
Every kernel still runs to its end in these cases (the loops of the
factorisations are bounded, comparisons with NaN skip rotations); the
argument errors that return before anything is enqueued are covered on the
host by tests/test_abi_host.py.
"""
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


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_nonfinite_theta_is_reported():
    dev = _dev()
    import paper_2409_05285_amd as p
    _say("NaN in theta")
    desc = p.Desc(4, 4, 2, 4)
    th = synth.theta_random_unit(4, 4, 2, 2, seed=5)
    th[:16] = np.nan                                  # site 0: d^2 slices of 1 x 1 x 2 x 2
    cfg = torch.tensor(synth.configs_sector(3, 16, 2, seed=6), device=dev)
    la, sg, el, st = p.peps_eval_batch(desc, torch.tensor(th, device=dev), cfg)
    torch.cuda.synchronize()
    with pytest.raises(p.PepsError) as e:
        p.check(st)
    assert e.value.code == -5


def test_zero_amplitude_is_reported():
    dev = _dev()
    import paper_2409_05285_amd as p
    _say("zero amplitude")
    desc = p.Desc(4, 4, 2, 4)
    th = torch.tensor(synth.theta_identity(4, 4, 2, 2), device=dev)
    cfg = synth.configs_diagonal(2, 16, 2, seed=6)
    cfg[1, 5] = 2 * (cfg[1, 5] // 2) + (1 - cfg[1, 5] // 2)   # s != s' at site 5 of sample 1
    la, sg, el, st = p.peps_eval_batch(desc, th, torch.tensor(cfg, device=dev))
    torch.cuda.synchronize()
    with pytest.raises(p.PepsError) as e:
        p.check(st)
    assert e.value.code == -6
    la = la.cpu().numpy()
    assert abs(la[0]) < 1e-12 and np.isneginf(la[1])
    res = p.peps_sample_sweep(desc, th, torch.tensor(cfg, device=dev), 3, 0, 1)
    torch.cuda.synchronize()
    with pytest.raises(p.PepsError) as e:
        p.check(res["status"])
    assert e.value.code == -6


def _step(p, desc, theta, configs, seed, sweep0, S):
    res = p.peps_sample_sweep(desc, theta, configs, seed, sweep0, S, want_configs=True)
    n = configs.shape[0]
    nnz = p.peps_orow_count(desc)
    _, _, _, st = p.sr_cg_solve(desc, res["configs"].reshape(S * n, desc.N), res["O"].reshape(S * n, nnz),
                                res["e_loc"].reshape(S * n), 0.02, 1e-4, 50, 1e-10, want_g=False, theta=theta)
    torch.cuda.synchronize()
    p.check(res["status"])
    p.check(st)
    return sweep0 + S


@pytest.mark.parametrize("mixed", [False, True])
def test_resume_from_saved_state_is_bit_exact(mixed, tmp_path):
    dev = _dev()
    import paper_2409_05285_amd as p
    _say("resume", "mixed" if mixed else "fp64")
    desc = p.Desc(4, 4, 2, 4, precision=p.PREC_MIXED if mixed else p.PREC_FP64)
    th0 = synth.theta_identity(4, 4, 2, 2, noise=1e-2, seed=11)
    cfg0 = synth.configs_diagonal(32, 16, 2, seed=12)
    seed, S = 4242, 3
    th_a = torch.tensor(th0, device=dev)
    cfg_a = torch.tensor(cfg0, device=dev)
    g = _step(p, desc, th_a, cfg_a, seed, 0, S)
    _step(p, desc, th_a, cfg_a, seed, g, S)
    th_b = torch.tensor(th0, device=dev)
    cfg_b = torch.tensor(cfg0, device=dev)
    g = _step(p, desc, th_b, cfg_b, seed, 0, S)
    path = tmp_path / "state.npz"
    np.savez(path, theta=th_b.cpu().numpy(), configs=cfg_b.cpu().numpy(), gsweep=g)
    del th_b, cfg_b
    st = np.load(path)
    th_c = torch.tensor(st["theta"], device=dev)
    cfg_c = torch.tensor(st["configs"], device=dev)
    _step(p, desc, th_c, cfg_c, seed, int(st["gsweep"]), S)
    assert torch.equal(th_a, th_c)
    assert torch.equal(cfg_a, cfg_c)
    assert not np.array_equal(th_a.cpu().numpy(), th0)
