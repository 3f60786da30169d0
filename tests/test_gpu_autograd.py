"""The adjoint path on the GPU: PepsLogAmp (forward peps_grad_batch, backward
peps_vjp_batch) against the oracle's O rows and central finite differences.

Bar: the backward of sum_i c_i log|psi_i| matches sum_i c_i O_i of the
oracle within 1e-9 (relative to the largest entry).  Where chi is exact the
boundary MPS does not depend on theta through a truncation, O is then the
true gradient of log|psi|, and central differences of the oracle's log|psi|
(h = 1e-6, FP64) on sampled parameters agree within 1e-6 relative (the
amplitude is linear in each tensor entry, so the central difference has no
truncation error beyond round-off).  With truncation O is the derivative of
the row strip with its boundaries held fixed (Eq. 8 under truncation), which
is what the backward returns.
"""
import numpy as np
import pytest

import synth
from oracle import measure, sr
from oracle.lattice import Lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


@pytest.mark.parametrize("L1,L2,D,chi,exact", [(3, 3, 2, 4, True), (4, 4, 2, 4, True), (4, 5, 3, 5, False)])
def test_logamp_backward_matches_oracle(L1, L2, D, chi, exact):
    dev = _dev()
    import paper_2409_05285_amd as p
    lat = Lattice(L1, L2, D=D, chi=chi)
    desc = p.Desc(L1, L2, D, chi)
    th = synth.theta_random_unit(L1, L2, D, 2, seed=31)
    cfg = synth.configs_sector(4, lat.N, 2, seed=32)
    coef = np.array([0.7, -1.3, 0.4, 2.0])
    print("[case] autograd", L1, L2, D, chi, flush=True)
    theta = torch.tensor(th, device=dev, requires_grad=True)
    la = p.PepsLogAmp.apply(theta, torch.tensor(cfg, device=dev), desc)
    (la * torch.tensor(coef, device=dev)).sum().backward()
    grad = theta.grad.cpu().numpy()
    ref = measure.evaluate_batch(lat, th, cfg, chi)
    np.testing.assert_allclose(la.detach().cpu().numpy(), ref["log_abs"], rtol=1e-10, atol=1e-10)
    expect = sr.dense_O(lat, cfg, ref["O"]).T @ coef
    assert np.all(np.abs(grad - expect) <= 1e-9 * np.abs(expect).max())
    if not exact:
        return
    # central differences of the oracle's log|psi| on a few parameters
    rng = np.random.default_rng(33)
    h = 1e-6
    for k in rng.choice(lat.n_params, size=12, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fp = measure.evaluate_batch(lat, tp, cfg, chi, want_O=False)["log_abs"] @ coef
        fm = measure.evaluate_batch(lat, tm, cfg, chi, want_O=False)["log_abs"] @ coef
        fd = (fp - fm) / (2 * h)
        assert abs(grad[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, grad[k], fd)


def test_vjp_matches_sum_of_rows_8x8():
    """At the 8x8, D=4, chi=16 shape: the device VJP against the oracle's
    expansion of the device's own O rows (checks the scatter alone)."""
    dev = _dev()
    import paper_2409_05285_amd as p
    lat = Lattice(8, 8, D=4, chi=16)
    desc = p.Desc(8, 8, 4, 16)
    th = synth.theta_random_unit(8, 8, 4, 2, seed=34)
    cfg = synth.configs_sector(64, lat.N, 2, seed=35)
    cot = np.random.default_rng(36).standard_normal(64)
    print("[case] vjp 8x8", flush=True)
    cfg_d = torch.tensor(cfg, device=dev)
    O, la, st = p.peps_grad_batch(desc, torch.tensor(th, device=dev), cfg_d)
    grad = p.peps_vjp_batch(desc, cfg_d, O, torch.tensor(cot, device=dev))
    torch.cuda.synchronize()
    assert p.check(st) == 0
    expect = sr.dense_O(lat, cfg, O.cpu().numpy()).T @ cot
    assert np.all(np.abs(grad.cpu().numpy() - expect) <= 1e-12 * np.abs(expect).max())
