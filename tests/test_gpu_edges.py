"""Edge cases of the device path against the oracle: the smallest lattice,
bond dimension 1 (product states), boundary dimension 1 (every cut truncated
to one value), the widest row (L2 = 32) and the largest site count
(L1 L2 = 256); and empty batches for every entry point (no-ops).
Bars as in the other FP64 parity tests."""
import sys

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
