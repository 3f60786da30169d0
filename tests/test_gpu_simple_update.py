"""Simple update on the device against the oracle's simple update.

Both sides start from the same random PEPS with all bond weights 1 and run
the same steps.  Their bond gauges differ (QR versus Jacobi factors, signs of
singular vectors), so only gauge-invariant results are compared: the bond
weights (normalised singular values) to 1e-10, and the amplitudes of the
absorbed PEPS, from the device's own evaluation (chi large enough to be
exact) against the oracle's exact contraction of its own result, to 1e-10
in log|psi| with equal signs.  The step is also timed on both sides."""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import network
from oracle import simple_update as su
from oracle.lattice import Lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


@pytest.mark.parametrize("L1,L2,D,start", [(4, 4, 2, "random"), (3, 4, 3, "random"), (4, 4, 4, "random"),
                                           (4, 4, 4, "identity"), (3, 3, 6, "random"), (3, 3, 8, "random")])
def test_simple_update_matches_oracle(L1, L2, D, start):
    dev = _dev()
    import paper_2409_05285_amd as p
    print("[case] simple update", L1, L2, D, start, flush=True)
    sys.stdout.flush()
    chi = D * D
    lat = Lattice(L1, L2, D=D, chi=chi)
    desc = p.Desc(L1, L2, D, chi)
    if start == "random":
        th = synth.theta_random_unit(L1, L2, D, 2, seed=91)
    else:
        th = synth.theta_identity(L1, L2, D, 2, noise=1e-2, seed=92)
    nb = p.su_bond_count(desc)
    steps, tau = 3, 0.05
    th_d = torch.tensor(th, device=dev)
    lam_d = torch.ones((nb, D), dtype=torch.float64, device=dev)
    st = p.peps_simple_update(desc, th_d, lam_d, tau, steps)
    abs_d = p.peps_su_absorb(desc, th_d, lam_d)
    torch.cuda.synchronize()
    assert p.check(st) == 0
    th_o = th.copy()
    lam_o = np.ones((nb, D))
    for _ in range(steps):
        su.su_step(lat, th_o, lam_o, tau)
    abs_o = su.absorb(lat, th_o, lam_o)
    lam_dev = lam_d.cpu().numpy()
    assert np.all(np.abs(lam_dev - lam_o) <= 1e-10), np.abs(lam_dev - lam_o).max()
    cfg = synth.configs_sector(8, lat.N, 2, seed=93) if start == "random" else \
        synth.configs_diagonal(8, lat.N, 2, seed=94)
    la, sg, _, st2 = p.peps_eval_batch(desc, abs_d, torch.tensor(cfg, device=dev), want_e=False)
    torch.cuda.synchronize()
    assert p.check(st2) == 0
    la, sg = la.cpu().numpy(), sg.cpu().numpy()
    amp = np.array([network.amplitude(lat, abs_o, S) for S in cfg])
    assert np.all(np.abs(la - np.log(np.abs(amp))) <= 1e-10 * np.maximum(1.0, np.abs(la))), (la, np.log(np.abs(amp)))
    assert np.array_equal(sg, np.sign(amp).astype(np.int8))


def test_simple_update_step_time():
    """Time of one step on the 8 x 8 lattice at D = 4 (device, 100 steps) and
    in the oracle (one step); printed, and the device result checked finite."""
    dev = _dev()
    import paper_2409_05285_amd as p
    print("[case] simple update timing 8x8 D=4", flush=True)
    desc = p.Desc(8, 8, 4, 16)
    lat = Lattice(8, 8, D=4, chi=16)
    th = synth.theta_identity(8, 8, 4, 2, noise=1e-2, seed=95)
    nb = p.su_bond_count(desc)
    th_d = torch.tensor(th, device=dev)
    lam_d = torch.ones((nb, 4), dtype=torch.float64, device=dev)
    p.peps_simple_update(desc, th_d, lam_d, 0.01, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = p.peps_simple_update(desc, th_d, lam_d, 0.01, 100)
    torch.cuda.synchronize()
    t_dev = (time.perf_counter() - t0) / 100
    assert p.check(st) == 0
    assert torch.isfinite(th_d).all() and torch.isfinite(lam_d).all()
    th_o = th.copy()
    lam_o = np.ones((nb, 4))
    t0 = time.perf_counter()
    su.su_step(lat, th_o, lam_o, 0.01)
    t_cpu = time.perf_counter() - t0
    print("[time] simple-update step, 8x8 D=4 (112 bonds): device %.3f ms, oracle %.1f ms" % (t_dev * 1e3, t_cpu * 1e3),
          flush=True)
