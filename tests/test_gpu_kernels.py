"""The three boundary-compression kernels (register-, LDS- and
workspace-resident), each forced through peps_desc.compress_kernel on the
shapes where it applies, against the oracle at the FP64 bars: evaluation
and O rows (log|psi| and E_loc 1e-10, O 1e-9) and one sweep bit-exact; and
the autotuner that picks among them (peps_autotune_compression, with its
JSON cache)."""
import json
import sys

import numpy as np
import pytest

import synth
from oracle import measure, sampler
from oracle.lattice import Lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [(4, 4, 2, 4, 0.0), (4, 5, 3, 5, 0.0), (4, 4, 2, 3, 0.5), (3, 4, 4, 6, 0.0)]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("kernel", [1, 2, 3])
@pytest.mark.parametrize("L1,L2,D,chi,J2", SHAPES)
def test_forced_kernel_matches_oracle(L1, L2, D, chi, J2, kernel):
    import paper_2409_05285_amd as p
    dev = _dev()
    desc = p.Desc(L1, L2, D, chi, J2=J2, compress_kernel=kernel)
    lat = Lattice(L1, L2, D=D, chi=chi, J2=J2)
    th = synth.theta_random_unit(L1, L2, D, 2, seed=121)
    cfg = synth.configs_sector(3, L1 * L2, 2, seed=122)
    theta_d = torch.tensor(th, device=dev)
    try:
        la, sg, el, st = p.peps_eval_batch(desc, theta_d, torch.tensor(cfg, device=dev))
    except p.PepsError as e:
        assert e.code == -2
        pytest.skip("kernel not applicable to this shape")
    _say("forced compression kernel", kernel, L1, L2, D, chi, J2)
    O, _, st2 = p.peps_grad_batch(desc, theta_d, torch.tensor(cfg, device=dev))
    torch.cuda.synchronize()
    assert p.check(st) == 0 and p.check(st2) == 0
    ref = measure.evaluate_batch(lat, th, cfg, chi)
    la, sg, el, O = (x.cpu().numpy() for x in (la, sg, el, O))
    emag = max(np.abs(ref["e_loc"]).mean(), 1e-300)
    assert np.all(np.abs(la - ref["log_abs"]) <= 1e-10 * np.maximum(1.0, np.abs(ref["log_abs"])))
    assert np.array_equal(sg, ref["sign"])
    assert np.all(np.abs(el - ref["e_loc"]) <= 1e-10 * np.maximum(np.abs(ref["e_loc"]), emag))
    assert np.all(np.abs(O - ref["O"]) <= 1e-9 * np.maximum(1.0, np.abs(ref["O"])))
    # one sweep of two chains, bit-exact against the oracle's sweep
    c0 = synth.configs_diagonal(2, L1 * L2, 2, seed=123)
    cd = torch.tensor(c0, device=dev)
    res = p.peps_sample_sweep(desc, theta_d, cd, 31, 0, 1, measure=False)
    torch.cuda.synchronize()
    assert p.check(res["status"]) == 0
    got, acc = cd.cpu().numpy(), res["n_accept"].cpu().numpy()
    for ch in range(2):
        r = sampler.sweep(lat, th, c0[ch].astype(np.int64), chi, 31, ch, 0, tie_tol=1e-12)
        if r["near_ties"]:
            continue
        assert np.array_equal(got[ch], r["S"].astype(np.uint8)) and np.array_equal(acc[ch], r["n_accept"])


def test_autotuner_picks_a_valid_kernel_and_caches_it(tmp_path):
    import paper_2409_05285_amd as p
    dev = _dev()
    _say("compression autotuner")
    desc = p.Desc(4, 4, 2, 4, precision=p.PREC_MIXED)
    th = torch.tensor(synth.theta_random_unit(4, 4, 2, 2, seed=124), device=dev)
    cfg = torch.tensor(synth.configs_diagonal(256, 16, 2, seed=125), device=dev)
    cache = str(tmp_path / "tune.json")
    tuned, rec = p.tune_compression(desc, th, cfg, cache_path=cache)
    assert not rec["cached"] and set(rec["ms"]) == {"register", "lds", "workspace"}
    assert all(v > 0.0 for v in rec["ms"].values())
    assert rec["best"] == min(rec["ms"], key=rec["ms"].get)
    assert tuned.compress_kernel in (1, 2, 3)
    stored = json.load(open(cache))
    assert list(stored.values())[0]["best"] == rec["best"]
    tuned2, rec2 = p.tune_compression(desc, th, cfg, cache_path=cache)
    assert rec2["cached"] and tuned2 == tuned
    # the tuned descriptor evaluates like the automatic one, to rounding
    la1, _, e1, s1 = p.peps_eval_batch(desc, th, cfg)
    la2, _, e2, s2 = p.peps_eval_batch(tuned, th, cfg)
    torch.cuda.synchronize()
    assert p.check(s1) == 0 and p.check(s2) == 0
    assert torch.allclose(la1, la2, rtol=1e-4, atol=1e-4)
