"""The instrumentation handle: per-class launch times and counts, and the
progress hook that reports each traced launch as it completes (the
library's stderr printer)."""
import sys

import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_trace_counts_and_progress_lines(capfd):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2409_05285_amd as p
    print("[case] trace and progress hook", flush=True)
    sys.stdout.flush()
    dev = torch.device("cuda:0")
    desc = p.Desc(4, 4, 2, 4)
    th = torch.tensor(synth.theta_random_unit(4, 4, 2, 2, seed=3), device=dev)
    cfg = torch.tensor(synth.configs_diagonal(8, 16, 2, seed=4), device=dev)
    tr = p.Trace(256)
    tr.on_progress("eval 4x4")
    p.peps_eval_batch(desc, th, cfg, trace=tr)
    torch.cuda.synchronize()
    prof = tr.read()
    tr.on_progress(None)
    p.peps_eval_batch(desc, th, cfg, trace=tr)
    torch.cuda.synchronize()
    prof2 = tr.read()
    tr.close()
    err = capfd.readouterr().err
    lines = [x for x in err.splitlines() if x.startswith("[peps] eval 4x4 ")]
    n = sum(v[1] for v in prof.values())
    # 3 top and 3 bottom compressions, 4 one-row and 3 two-row measurements, finalisation
    assert prof["compress"][1] == 6 and prof["meas1"][1] == 4 and prof["meas2"][1] == 3 and prof["final"][1] == 1
    assert len(lines) == n, (len(lines), n)
    assert lines[0].startswith("[peps] eval 4x4 class 0 launch 0 done (")
    assert all(f"launch {i} done" in x for i, x in enumerate(lines))
    # the hook removed: the same counts, no more lines
    assert {k: v[1] for k, v in prof2.items()} == {k: v[1] for k, v in prof.items()}
    assert all(v[0] > 0.0 for v in prof.values() if v[1] > 0)
