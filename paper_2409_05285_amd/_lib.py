"""ctypes binding of libpeps.so (the C ABI declared in include/peps.h).

Argument marshalling only: tensors are torch tensors on the current HIP
device, passed by data pointer together with torch's current stream; every
step of the computation runs in the library's kernels.  Importing this
module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int8, c_int32, c_int64, c_size_t, c_uint8, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpeps.so")

PEPS_OK = 0
STATUS = {
    0: "ok", -1: "invalid argument or shape", -2: "unsupported by the device path", -3: "HIP failure",
    -4: "workspace too small", -5: "non-finite value", -6: "zero strip amplitude", -7: "CG breakdown",
    1: "CG not converged",
}
STATUS_HIP = -3
MODEL_HEISENBERG, MODEL_HUBBARD = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
WS_EVAL, WS_GRAD, WS_SWEEP, WS_SR, WS_SU, WS_MIN = 0, 1, 2, 3, 4, 5
COMPRESS_AUTO, COMPRESS_REGISTER, COMPRESS_LDS, COMPRESS_WORKSPACE = 0, 1, 2, 3
COMPRESS_NAMES = {1: "register", 2: "lds", 3: "workspace"}
N_OBS = 4   # peps_observables_batch: M_z, M_z^2, particle number, double occupancy


class PepsDesc(ctypes.Structure):
    _fields_ = [
        ("L1", c_int32), ("L2", c_int32), ("d", c_int32), ("D", c_int32), ("chi", c_int32),
        ("model", c_int32),
        ("J1", c_double), ("J2", c_double), ("t", c_double), ("U", c_double), ("mu", c_double),
        ("precision", c_int32), ("alpha", c_int32), ("fermionic", c_int32), ("compress_kernel", c_int32),
    ]


class PepsError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {STATUS.get(code, 'unknown')} (status {code})")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2409_05285_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P = POINTER(PepsDesc)
    lib.peps_param_count.argtypes = [P]
    lib.peps_param_count.restype = c_int64
    lib.peps_orow_count.argtypes = [P]
    lib.peps_orow_count.restype = c_int64
    lib.peps_slot_count.argtypes = [P]
    lib.peps_slot_count.restype = c_int64
    lib.peps_workspace_bytes.argtypes = [P, c_int64, c_int32, POINTER(c_size_t)]
    lib.peps_workspace_bytes.restype = c_int32
    lib.peps_status_string.argtypes = [c_int32]
    lib.peps_status_string.restype = ctypes.c_char_p
    lib.peps_eval_batch.argtypes = [P, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_size_t, c_void_p, c_void_p]
    lib.peps_eval_batch.restype = c_int32
    lib.peps_grad_batch.argtypes = [P, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_size_t, c_void_p, c_void_p]
    lib.peps_grad_batch.restype = c_int32
    lib.peps_sample_sweep.argtypes = [P, c_void_p, c_int32, c_void_p, c_uint64, c_uint64, c_void_p, c_int32, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_size_t, c_void_p, c_void_p]
    lib.peps_sample_sweep.restype = c_int32
    lib.sr_cg_solve.argtypes = [P, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double,
                                c_int32, c_double, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_size_t, c_void_p, c_void_p]
    lib.sr_cg_solve.restype = c_int32
    lib.peps_vjp_batch.argtypes = [P, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    lib.peps_vjp_batch.restype = c_int32
    lib.peps_observables_batch.argtypes = [P, c_int64, c_void_p, c_void_p, c_void_p]
    lib.peps_observables_batch.restype = c_int32
    lib.peps_simple_update.argtypes = [P, c_void_p, c_void_p, c_double, c_int32, c_void_p, c_void_p, c_size_t,
                                       c_void_p]
    lib.peps_simple_update.restype = c_int32
    lib.peps_su_absorb.argtypes = [P, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.peps_su_absorb.restype = c_int32
    lib.sr_cg_solve_noalloc.argtypes = [P, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                        c_double, c_int32, c_double, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_void_p]
    lib.sr_cg_solve_noalloc.restype = c_int32
    lib.peps_sample_stats.argtypes = [P, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p]
    lib.peps_sample_stats.restype = c_int32
    lib.peps_direct_workspace_bytes.argtypes = [P, c_int64, c_int32, POINTER(c_size_t)]
    lib.peps_direct_workspace_bytes.restype = c_int32
    lib.peps_direct_sample.argtypes = [P, c_void_p, c_int32, c_int32, c_uint64, c_uint64, c_int32, c_void_p, c_int32,
                                       c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]
    lib.peps_direct_sample.restype = c_int32
    lib.peps_importance_weights.argtypes = [c_int64, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.peps_importance_weights.restype = c_int32
    lib.peps_autotune_compression.argtypes = [P, c_void_p, c_int32, c_void_p, c_int32, POINTER(c_double),
                                              POINTER(c_int32), c_void_p, c_void_p, c_size_t, c_void_p]
    lib.peps_autotune_compression.restype = c_int32
    lib.peps_trace_create.argtypes = [c_int32]
    lib.peps_trace_create.restype = c_void_p
    lib.peps_trace_destroy.argtypes = [c_void_p]
    lib.peps_trace_destroy.restype = None
    lib.peps_trace_read.argtypes = [c_void_p, POINTER(c_double), POINTER(c_int64)]
    lib.peps_trace_read.restype = c_int32
    lib.peps_trace_set_progress.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.peps_trace_set_progress.restype = c_int32
    lib.peps_progress_stderr.argtypes = [c_void_p, c_int32, c_int32]
    lib.peps_progress_stderr.restype = None
    return lib


LIB = _load()
EXPORTS = ["peps_param_count", "peps_orow_count", "peps_slot_count", "peps_workspace_bytes",
           "peps_status_string", "peps_eval_batch", "peps_grad_batch", "peps_sample_sweep", "sr_cg_solve",
           "sr_cg_solve_noalloc",
           "peps_vjp_batch", "peps_observables_batch", "peps_sample_stats", "peps_simple_update",
           "peps_su_absorb", "peps_autotune_compression", "peps_direct_workspace_bytes", "peps_direct_sample", "peps_importance_weights",
           "peps_trace_create", "peps_trace_destroy", "peps_trace_read", "peps_trace_set_progress",
           "peps_progress_stderr"]
SR_STATIC_BYTES = 64 << 20   # scratch of sr_cg_solve_noalloc per GPU
SR_NSTATS = 5   # sr_cg_solve stats: Ebar, |r|, iterations, |b|, not-converged flag
KCLASS = ["compress", "moves1", "moves2", "meas1", "meas2", "final", "sr", "direct"]
