"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol include/peps.h declares, and its pure host queries agree with
the oracle's packing and reject bad descriptors."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "peps.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("peps_", "sr_"))))


def test_library_exports_every_declared_symbol():
    import paper_2409_05285_amd._lib as L
    lib = ctypes.CDLL(L.LIB_PATH)
    declared = _declared()
    assert set(declared) >= {"peps_eval_batch", "peps_grad_batch", "peps_sample_sweep", "sr_cg_solve"}
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(L.EXPORTS) == declared


@pytest.mark.parametrize("L1,L2,D,chi,d,model", [(4, 4, 2, 4, 2, 0), (8, 8, 4, 16, 2, 0), (3, 5, 3, 7, 2, 0),
                                                  (2, 3, 2, 4, 4, 1)])
def test_counts_match_oracle_packing(L1, L2, D, chi, d, model):
    import paper_2409_05285_amd as p
    from oracle.lattice import Lattice
    lat = Lattice(L1, L2, D=D, chi=chi, d=d, model=model)
    desc = p.Desc(L1, L2, D, chi, d=d, model=model)
    assert p.peps_param_count(desc) == lat.n_params
    assert p.peps_orow_count(desc) == lat.nnz
    assert p.peps_slot_count(desc) == lat.n_slots()


def test_workspace_and_errors():
    import paper_2409_05285_amd as p
    from paper_2409_05285_amd._lib import LIB
    desc = p.Desc(8, 8, 4, 16)
    a = p.peps_workspace_bytes(desc, 1, 2)
    b = p.peps_workspace_bytes(desc, 10, 2)
    assert b == 10 * a and a > 0
    assert p.peps_workspace_bytes(desc, 0, 0) == 0
    assert p.peps_workspace_bytes(desc, 100, 3) > 100 * 8
    with pytest.raises(p.PepsError):
        p.peps_workspace_bytes(desc, 5, 9)
    bad = p.Desc(1, 8, 4, 16)
    with pytest.raises(p.PepsError):
        p.peps_param_count(bad)
    with pytest.raises(p.PepsError):
        p.peps_param_count(p.Desc(4, 4, 2, 4, d=3))
    assert LIB.peps_status_string(-6) == b"zero strip amplitude for a sample"
    # device entry points reject bad descriptors before touching any pointer
    bd = bad.c()
    assert LIB.peps_eval_batch(ctypes.byref(bd), None, 1, None, None, None, None, None, None, 0, None, None) == -1
    # a valid call with n = 0 is a no-op that needs no device
    ok = desc.c()
    assert LIB.peps_eval_batch(ctypes.byref(ok), None, 0, None, None, None, None, None, None, 0, None, None) == 0
    # shapes beyond the compiled limits (chi * D > 512, or chi > 255) are refused
    big = p.Desc(4, 4, 8, 72).c()
    assert LIB.peps_eval_batch(ctypes.byref(big), None, 1, None, None, None, None, None, None, 0, None, None) == -2
    big = p.Desc(4, 4, 1, 256).c()
    assert LIB.peps_eval_batch(ctypes.byref(big), None, 1, None, None, None, None, None, None, 0, None, None) == -2
    # chi * D = 512 is within them: with n = 0 the call is a no-op
    edge = p.Desc(4, 4, 8, 64).c()
    assert LIB.peps_eval_batch(ctypes.byref(edge), None, 0, None, None, None, None, None, None, 0, None, None) == 0
    # the Hubbard model (d = 4) is accepted: with n = 0 the call is a no-op
    hub = p.Desc(2, 2, 2, 4, d=4, model=1).c()
    assert LIB.peps_eval_batch(ctypes.byref(hub), None, 0, None, None, None, None, None, None, 0, None, None) == 0
    # workspace too small
    assert LIB.peps_eval_batch(ctypes.byref(ok), ctypes.c_void_p(8), 1, ctypes.c_void_p(8), ctypes.c_void_p(8),
                               ctypes.c_void_p(8), None, None, ctypes.c_void_p(8), 16, None, None) == -4


def test_simple_update_entry_points_refuse_unsupported_cases():
    """The simple update covers the spin-1/2 Heisenberg model with J2 = 0 and
    D <= 8: other descriptors are refused before any pointer is touched; its
    workspace query scales with the largest bond group."""
    import paper_2409_05285_amd as p
    from paper_2409_05285_amd._lib import LIB
    ok = p.Desc(4, 4, 2, 4)
    assert p.peps_workspace_bytes(ok, 0, 4) > 0
    assert p.peps_workspace_bytes(p.Desc(8, 8, 2, 4), 0, 4) > p.peps_workspace_bytes(ok, 0, 4)
    for bad, code in ((p.Desc(4, 4, 2, 4, d=4, model=1), -2), (p.Desc(4, 4, 2, 4, J2=0.5), -2),
                      (p.Desc(4, 4, 9, 9), -2)):
        c = bad.c()
        assert LIB.peps_simple_update(ctypes.byref(c), None, None, 0.01, 1, None, None, 0, None) == code
        assert LIB.peps_su_absorb(ctypes.byref(c), None, None, None, None) == code
    c = ok.c()
    # zero steps is a no-op; missing buffers and a short workspace are argument errors
    assert LIB.peps_simple_update(ctypes.byref(c), None, None, 0.01, 0, None, None, 0, None) == 0
    assert LIB.peps_simple_update(ctypes.byref(c), None, None, 0.01, 1, None, None, 0, None) == -1
    assert LIB.peps_simple_update(ctypes.byref(c), ctypes.c_void_p(8), ctypes.c_void_p(8), 0.01, 1, None,
                                  ctypes.c_void_p(8), 16, None) == -4
    assert LIB.peps_simple_update(ctypes.byref(c), None, None, float("nan"), 1, None, None, 0, None) == -1


def test_binding_refuses_out_of_range_digits_and_bad_fermionic_flag():
    """Configuration digits must lie in [0, d^2): the binding refuses others
    before any launch (the device kernels check as well).  The fermionic
    flag is 0 or 1 and only for the Hubbard model."""
    import torch

    import paper_2409_05285_amd as p
    desc = p.Desc(4, 4, 2, 4)
    th = torch.zeros(p.peps_param_count(desc), dtype=torch.float64)
    cfg = torch.zeros((2, 16), dtype=torch.uint8)
    cfg[1, 3] = 4
    with pytest.raises(ValueError):
        p.peps_eval_batch(desc, th, cfg)
    hub = p.Desc(4, 4, 2, 4, d=4, model=1)
    cfg[1, 3] = 16
    with pytest.raises(ValueError):
        p.peps_grad_batch(hub, torch.zeros(p.peps_param_count(hub), dtype=torch.float64), cfg)
    assert p.peps_param_count(p.Desc(4, 4, 2, 4, d=4, model=1, fermionic=1)) > 0
    for bad in (p.Desc(4, 4, 2, 4, fermionic=1), p.Desc(4, 4, 2, 4, d=4, model=1, fermionic=2)):
        with pytest.raises(p.PepsError):
            p.peps_param_count(bad)


def test_noalloc_solve_refuses_sizes_beyond_its_scratch():
    """sr_cg_solve_noalloc checks its fixed scratch (64 MiB per GPU) against
    the workspace the problem needs and returns PEPS_ERR_WORKSPACE (-4)
    before anything is enqueued or any device call is made; bad arguments
    give PEPS_ERR_ARG (-1) the same way."""
    import paper_2409_05285_amd as p
    from paper_2409_05285_amd._lib import LIB, SR_STATIC_BYTES
    desc = p.Desc(16, 16, 8, 64)
    n_s = 512
    assert p.peps_workspace_bytes(desc, n_s, 3) > SR_STATIC_BYTES
    c = desc.c()
    v = ctypes.c_void_p(8)
    assert LIB.sr_cg_solve_noalloc(ctypes.byref(c), n_s, v, v, None, None, v, 0.01, 1e-4, 10, 0.0, v, None, None, v,
                                   None, None) == -4
    assert LIB.sr_cg_solve_noalloc(ctypes.byref(c), 0, v, v, None, None, v, 0.01, 1e-4, 10, 0.0, v, None, None, v,
                                   None, None) == -1
    assert LIB.sr_cg_solve_noalloc(ctypes.byref(c), n_s, None, v, None, None, v, 0.01, 1e-4, 10, 0.0, v, None, None,
                                   v, None, None) == -1


def test_smallest_workspace_layout():
    """Where the QR matrices do not fit on chip (chi * D > 64) the smallest
    accepted workspace keeps R factors instead of every site's reflectors:
    at 16x16, D = 8, chi = 64 it is well under the full size, elsewhere the
    two sizes are equal; a workspace between the two is accepted, one below
    the smallest is refused (with n = 0 no size is needed)."""
    import paper_2409_05285_amd as p
    from paper_2409_05285_amd._lib import LIB, WS_MIN
    big = p.Desc(16, 16, 8, 64)
    full, small = p.peps_workspace_bytes(big, 4, 2), p.peps_workspace_bytes(big, 4, WS_MIN)
    assert small < 0.6 * full
    for d in (p.Desc(8, 8, 4, 16), p.Desc(4, 4, 2, 4), p.Desc(4, 4, 3, 7)):
        assert p.peps_workspace_bytes(d, 4, WS_MIN) == p.peps_workspace_bytes(d, 4, 2)
    c = big.c()
    v = ctypes.c_void_p(8)
    assert LIB.peps_eval_batch(ctypes.byref(c), v, 4, v, v, v, None, None, v, small - 8, None, None) == -4


def test_direct_sampling_entry_points_check_their_arguments():
    """peps_direct_sample / peps_direct_workspace_bytes / peps_importance_weights
    return argument, size and support errors before enqueuing anything."""
    import paper_2409_05285_amd as p
    from paper_2409_05285_amd._lib import LIB
    desc = p.Desc(4, 4, 2, 4)
    c = desc.c()
    a = p.peps_direct_workspace_bytes(desc, 1, 16)
    b = p.peps_direct_workspace_bytes(desc, 9, 16)
    assert a > 0 and b > a
    assert p.peps_direct_workspace_bytes(desc, 0, 16) < a
    with pytest.raises(p.PepsError):
        p.peps_direct_workspace_bytes(desc, 1, 0)
    with pytest.raises(p.PepsError):     # D^6 chi^2 chi_dl intermediates beyond the kernel's limit
        p.peps_direct_workspace_bytes(p.Desc(6, 6, 4, 16), 1, 64)
    v = ctypes.c_void_p(0x1000)
    call = lambda n, chi_dl, rw, bd, ub, ws_bytes, reuse=0: LIB.peps_direct_sample(
        ctypes.byref(c), v, n, chi_dl, 1, 0, rw, bd, ub, reuse, v, v, v, v, ws_bytes, None, None)
    assert call(-1, 16, 0, None, 0, 1 << 40) == -1
    assert call(4, 0, 0, None, 0, 1 << 40) == -1
    assert call(4, 16, 2, None, 0, 1 << 40) == -1
    assert call(4, 16, 1, None, 0, 1 << 40) == -1      # reweighting needs b_diag
    assert call(4, 16, 0, None, 1, 1 << 40) == -1      # so does its update
    assert call(4, 16, 0, None, 0, 1000) == -4         # workspace too small
    assert call(4, 16, 0, None, 0, 1 << 40, 2) == -1   # reuse flag is 0 or 1
    assert call(0, 16, 0, None, 0, 0) == 0             # nothing to draw
    assert LIB.peps_importance_weights(0, v, v, v, None) == -1
    assert LIB.peps_importance_weights(5, None, v, v, None) == -1


def test_compression_kernel_choice_is_validated():
    """peps_desc.compress_kernel: values outside 0..3 make the descriptor
    invalid; a forced kernel whose limits the shape exceeds is refused with
    PEPS_ERR_UNSUPPORTED before anything is enqueued; the workspace size
    follows the chosen kernel."""
    import paper_2409_05285_amd as p
    from paper_2409_05285_amd._lib import LIB
    with pytest.raises(p.PepsError):
        p.peps_param_count(p.Desc(4, 4, 2, 4, compress_kernel=4))
    a = p.peps_workspace_bytes(p.Desc(4, 4, 2, 4, compress_kernel=1), 8, 0)
    b = p.peps_workspace_bytes(p.Desc(4, 4, 2, 4, compress_kernel=3), 8, 0)
    assert a == p.peps_workspace_bytes(p.Desc(4, 4, 2, 4), 8, 0) and b > a
    v = ctypes.c_void_p(0x1000)
    for desc in (p.Desc(4, 4, 3, 5, compress_kernel=1),      # D = 3: no register kernel
                 p.Desc(6, 6, 4, 20, compress_kernel=2),     # chi D = 80 at D = 4: beyond the LDS kernel
                 p.Desc(6, 6, 4, 20, compress_kernel=1)):    # and beyond the register kernel
        c = desc.c()
        assert LIB.peps_eval_batch(ctypes.byref(c), v, 4, v, v, v, v, v, v, 1 << 40, None, None) == -2
