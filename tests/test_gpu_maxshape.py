"""Bond dimension D = 8 and the largest boundary shape the library accepts.

* 4x4, D = 8, chi = 16 (chi D = 128): evaluation, O rows and one sweep
  against the oracle, FP64 and mixed, at the bars of the other parity tests.
* 6x6, D = 8, chi = 64 (chi D = 512, the limit): the interior sites reach
  4096 x 512 QR matrices and 512-column truncations, so the workspace-resident
  kernel's streamed paths (QR columns and Jacobi columns longer than its
  register batches) run; evaluation and O rows of two samples in FP64 against
  the oracle, at the FP64 bars of every other lattice (1e-10 on log|psi| and
  E_loc, 1e-9 on O); the same for the Hubbard model (d^2 = 16, parity-even
  tensors).
"""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import measure, sampler
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


def _check(p, lat, desc, th, cfg, chi, tol_e, tol_o, mixed):
    dev = _dev()
    theta_d = torch.tensor(th, device=dev)
    cfg_d = torch.tensor(cfg, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    la, sg, el, st = p.peps_eval_batch(desc, theta_d, cfg_d)
    O, _, st2 = p.peps_grad_batch(desc, theta_d, cfg_d)
    torch.cuda.synchronize()
    print("[time] device eval + grad of %d samples: %.2f s" % (cfg.shape[0], time.perf_counter() - t0), flush=True)
    assert p.check(st) == 0 and p.check(st2) == 0
    ref = measure.evaluate_batch(lat, th, cfg, chi)
    la, sg, el, O = (x.cpu().numpy() for x in (la, sg, el, O))
    emag0 = max(np.abs(ref["e_loc"]).mean(), 1e-300)
    print("[err] log|psi| %.2e  E_loc %.2e  O %.2e" % (
        (np.abs(la - ref["log_abs"]) / np.maximum(1.0, np.abs(ref["log_abs"]))).max(),
        (np.abs(el - ref["e_loc"]) / np.maximum(np.abs(ref["e_loc"]), emag0)).max(),
        (np.abs(O - ref["O"]) / np.maximum(1.0, np.abs(ref["O"]))).max()), flush=True)
    assert np.all(np.abs(la - ref["log_abs"]) <= tol_e * np.maximum(1.0, np.abs(ref["log_abs"]))), (la, ref["log_abs"])
    assert np.array_equal(sg, ref["sign"])
    emag = max(np.abs(ref["e_loc"]).mean(), 1e-300)
    assert np.all(np.abs(el - ref["e_loc"]) <= tol_e * np.maximum(np.abs(ref["e_loc"]), emag)), (el, ref["e_loc"])
    if mixed:
        for i in range(O.shape[0]):
            assert np.all(np.abs(O[i] - ref["O"][i]) <= 1e-4 * np.abs(ref["O"][i]).max())
    else:
        assert np.all(np.abs(O - ref["O"]) <= tol_o * np.maximum(1.0, np.abs(ref["O"])))


@pytest.mark.parametrize("mixed", [False, True])
def test_bond_dimension_8(mixed):
    import paper_2409_05285_amd as p
    _say("4x4 D=8 chi=16", "mixed" if mixed else "fp64")
    lat = Lattice(4, 4, D=8, chi=16)
    desc = p.Desc(4, 4, 8, 16, precision=p.PREC_MIXED if mixed else p.PREC_FP64)
    th = synth.theta_random_unit(4, 4, 8, 2, seed=7)
    cfg = synth.configs_sector(3, 16, 2, seed=44)
    tol = 1e-4 if mixed else 1e-10
    _check(p, lat, desc, th, cfg, 16, tol, 1e-9, mixed)


def test_bond_dimension_8_sweep_bit_exact():
    dev = _dev()
    import paper_2409_05285_amd as p
    _say("4x4 D=8 chi=16 sweep")
    lat = Lattice(4, 4, D=8, chi=16)
    desc = p.Desc(4, 4, 8, 16)
    th = synth.theta_random_unit(4, 4, 8, 2, seed=7)
    cfg = synth.configs_diagonal(3, 16, 2, seed=45)
    cfg_d = torch.tensor(cfg, device=dev)
    res = p.peps_sample_sweep(desc, torch.tensor(th, device=dev), cfg_d, 5, 0, 1)
    torch.cuda.synchronize()
    assert p.check(res["status"]) == 0
    got = cfg_d.cpu().numpy()
    acc = res["n_accept"].cpu().numpy()
    compared = 0
    for ch in range(cfg.shape[0]):
        r = sampler.sweep(lat, th, cfg[ch].astype(np.int64), 16, 5, ch, 0, tie_tol=1e-12)
        if r["near_ties"]:
            continue
        compared += 1
        assert np.array_equal(got[ch], r["S"].astype(np.uint8)), ch
        assert np.array_equal(acc[ch], r["n_accept"]), ch
    assert compared >= 2


def test_largest_boundary_shape():
    import paper_2409_05285_amd as p
    _say("6x6 D=8 chi=64 (chi D = 512)")
    lat = Lattice(6, 6, D=8, chi=64)
    desc = p.Desc(6, 6, 8, 64)
    th = synth.theta_random_unit(6, 6, 8, 2, seed=7)
    cfg = synth.configs_sector(2, 36, 2, seed=46)
    _check(p, lat, desc, th, cfg, 64, 1e-10, 1e-9, False)


def test_hubbard_largest_boundary_shape():
    """The Hubbard lattice at the largest boundary shape: 6x6, d^2 = 16, D =
    8, chi = 64 (chi D = 512), t = 1, U = 8, mu = 4, Z2-graded parity-even
    tensors declared (fermionic = 1), two even-parity configurations (equal
    particle numbers in s and s'): FP64 evaluation and O rows against the
    oracle at the FP64 bars, Jordan-Wigner hop signs included."""
    import paper_2409_05285_amd as p
    from oracle.lattice import MODEL_HUBBARD
    _say("6x6 Hubbard D=8 chi=64 (chi D = 512)")
    hub = dict(t=1.0, U=8.0, mu=4.0)
    lat = Lattice(6, 6, D=8, chi=64, d=4, model=MODEL_HUBBARD, **hub)
    desc = p.Desc(6, 6, 8, 64, d=4, model=p.MODEL_HUBBARD, fermionic=1, **hub)
    th = synth.theta_random_parity_even(6, 6, 8, 4, seed=47)
    cfg = synth.configs_sector(2, 36, 4, seed=48)
    _check(p, lat, desc, th, cfg, 64, 1e-10, 1e-9, False)


def test_smallest_workspace_layout_is_bit_identical():
    """The workspace-resident compression in its two layouts -- every site's
    QR reflectors kept (full workspace) or rebuilt from the stored R factors
    (the smallest workspace, PEPS_WS_MIN) -- gives the same sweep, log|psi|,
    local energies and O rows bit for bit (6x6, D = 4, chi = 20: chi D = 80,
    past the on-chip kernels)."""
    dev = _dev()
    import paper_2409_05285_amd as p
    _say("workspace layouts, 6x6 D=4 chi=20")
    desc = p.Desc(6, 6, 4, 20, J2=0.5)
    th = torch.tensor(synth.theta_random_unit(6, 6, 4, 2, seed=81), device=dev)
    cfg0 = synth.configs_diagonal(8, 36, 2, seed=82)
    n = cfg0.shape[0]
    full, small = p.workspace_bytes(desc, n, "sweep"), p.workspace_bytes(desc, n, "min")
    assert small < full
    outs = []
    for nb in (full, small):
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        cfg = torch.tensor(cfg0, device=dev)
        res = p.peps_sample_sweep(desc, th, cfg, 77, 0, 2, ws=ws)
        torch.cuda.synchronize()
        assert p.check(res["status"]) == 0
        outs.append((cfg.cpu().numpy(), res["log_abs"].cpu().numpy(), res["e_loc"].cpu().numpy(),
                     res["O"].cpu().numpy()))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
