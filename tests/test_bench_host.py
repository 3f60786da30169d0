"""Host-side checks of bench.py (no GPU): more than one GPU is refused with
a message before anything touches a device, and the compression work model
it reports against agrees with a direct count for a lattice small enough to
count by hand."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_compression_model_small_case():
    """2x2 lattice, D = 1: every site matrix is 1 x 1 (absorption 2 flops,
    QR of 1 x 1, SVD of 1 x 1), so the model reduces to its per-site terms."""
    sys.path.insert(0, ROOT)
    import bench
    fl, dims = bench.compression_flops(2, 2, 1, 1, 0, 0, None)
    # absorption 2 a Dl p b Dr q = 2 per site; QR(1, 1) = 2 (2 - 2/3) each; R B = 2 - 1 = 1; SVD(1, 1) = 21;
    # B U S = 2 per site of the right-to-left sweep
    qr = 2 * (2 - 2 / 3)
    want = 2 * 2 + (qr + 1) + (21 + 2)
    assert abs(fl - want) < 1e-12
    assert dims == [(1, 1, 1), (1, 1, 1)]
