"""Python face of the C ABI, with the same names as include/peps.h.

Tensors live on the current HIP device (torch is used for device memory
and streams only).  Each call validates shapes, allocates outputs and a
cached workspace, and enqueues the library call on torch's current stream.
Device status words are returned as tensors; `check(status)` synchronises
and raises on a recorded failure.
"""
from __future__ import annotations

import ctypes
import dataclasses
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import LIB, PepsDesc, PepsError


@dataclass(frozen=True)
class Desc:
    """Problem descriptor (peps_desc)."""
    L1: int
    L2: int
    D: int
    chi: int
    d: int = 2
    model: int = _lib.MODEL_HEISENBERG
    J1: float = 1.0
    J2: float = 0.0
    t: float = 1.0
    U: float = 0.0
    mu: float = 0.0
    precision: int = _lib.PREC_FP64
    alpha: int = 2
    fermionic: int = 0
    compress_kernel: int = _lib.COMPRESS_AUTO

    def c(self):
        return PepsDesc(self.L1, self.L2, self.d, self.D, self.chi, self.model, self.J1, self.J2, self.t,
                        self.U, self.mu, self.precision, self.alpha, self.fermionic, self.compress_kernel)

    @property
    def N(self):
        return self.L1 * self.L2


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _raise(code, where):
    if code != _lib.PEPS_OK:
        raise PepsError(code, where)


def peps_param_count(desc: Desc) -> int:
    n = LIB.peps_param_count(ctypes.byref(desc.c()))
    _raise(0 if n >= 0 else -1, "peps_param_count")
    return int(n)


def peps_orow_count(desc: Desc) -> int:
    n = LIB.peps_orow_count(ctypes.byref(desc.c()))
    _raise(0 if n >= 0 else -1, "peps_orow_count")
    return int(n)


def peps_slot_count(desc: Desc) -> int:
    n = LIB.peps_slot_count(ctypes.byref(desc.c()))
    _raise(0 if n >= 0 else -1, "peps_slot_count")
    return int(n)


def peps_workspace_bytes(desc: Desc, n: int, what: int) -> int:
    out = ctypes.c_size_t(0)
    _raise(LIB.peps_workspace_bytes(ctypes.byref(desc.c()), int(n), int(what), ctypes.byref(out)),
           "peps_workspace_bytes")
    return int(out.value)


class Workspace:
    """Device workspace reused across calls (grown on demand)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes, device):
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = None   # release the old buffer before the new one is taken
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        return self.buf


_WS = {}


def _ws(kind, nbytes, device):
    w = _WS.setdefault(kind, Workspace())
    return w.get(nbytes, device)


def _own_ws(ws, kind, nbytes, device):
    """The caller's workspace after a size and device check, else the
    shared cache of that kind."""
    if ws is None:
        return _ws(kind, nbytes, device)
    if ws.dtype != torch.uint8 or not ws.is_contiguous() or ws.device != device or ws.numel() < max(int(nbytes), 256):
        raise ValueError("workspace must be a contiguous uint8 device tensor of at least %d bytes" % nbytes)
    return ws


def workspace_bytes(desc: Desc, n, kind):
    """Bytes of workspace a call on n chains ("sweep", "eval", "grad") or
    n_s samples ("sr") needs; "min": the smallest workspace an evaluation,
    gradient or sweep call on n chains accepts (the large-shape compression
    then rebuilds its QR reflectors instead of keeping them)."""
    what = {"sweep": _lib.WS_SWEEP, "eval": _lib.WS_EVAL, "grad": _lib.WS_GRAD, "sr": _lib.WS_SR,
            "min": _lib.WS_MIN}[kind]
    return peps_workspace_bytes(desc, n, what)


def _chain_ws(desc, n, what, device, ws=None):
    """The workspace of an evaluation, gradient or sweep call: the caller's
    (at least the smallest accepted size), else the shared cache, sized for
    the faster layout when the device has room for it and for the smallest
    one otherwise."""
    full = peps_workspace_bytes(desc, n, what)
    small = peps_workspace_bytes(desc, n, _lib.WS_MIN)
    if ws is not None:
        return _own_ws(ws, "chain", small, device)
    cur = _WS.get("chain")
    have = cur.buf.numel() if cur is not None and cur.buf is not None and cur.buf.device == device else 0
    if full > small and have < full:
        free, _ = torch.cuda.mem_get_info(device)
        if full - have > free - (1 << 30):
            return _ws("chain", small, device)
    return _ws("chain", full, device)


def _check_dev(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("tensors must be on the HIP device")


def _theta(desc, theta):
    if theta.dtype != torch.float64 or theta.dim() != 1 or theta.numel() != peps_param_count(desc):
        raise ValueError("theta must be a float64 vector of length N_p")
    return theta.contiguous()


def _configs(desc, configs):
    if configs.dtype != torch.uint8 or configs.dim() != 2 or configs.shape[1] != desc.N:
        raise ValueError("configs must be uint8 [n, L1*L2]")
    if not configs.is_contiguous():
        raise ValueError("configs must be contiguous")
    # digits must lie in [0, d^2); checked here unless a graph is being
    # captured (the library's kernels check on the device as well and record
    # PEPS_ERR_ARG in the status word)
    if configs.numel() > 0 and not (configs.is_cuda and torch.cuda.is_current_stream_capturing()):
        if int(configs.max()) >= desc.d * desc.d:
            raise ValueError("configuration digits must lie in [0, d^2)")
    return configs


class Trace:
    """Instrumentation handle (peps_trace): HIP events around the kernel
    launches of the calls it is passed to.  `read()` synchronises and returns
    {kernel class: (total ms, launches)} and empties the trace."""

    def __init__(self, capacity=1 << 16):
        self.h = LIB.peps_trace_create(int(capacity))
        if not self.h:
            raise PepsError(_lib.STATUS_HIP, "peps_trace_create")

    def read(self):
        ms = (ctypes.c_double * len(_lib.KCLASS))()
        cnt = (ctypes.c_int64 * len(_lib.KCLASS))()
        _raise(LIB.peps_trace_read(self.h, ms, cnt), "peps_trace_read")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(_lib.KCLASS)}

    def on_progress(self, label):
        """A line "[peps] <label> class <k> launch <i> done" on stderr as
        each traced launch completes (the library's own C printer, so the
        hook never enters Python while a thread may be waiting on the
        stream); None removes it."""
        if label is None:
            self._label = None
            _raise(LIB.peps_trace_set_progress(self.h, None, None), "peps_trace_set_progress")
            return
        self._label = ctypes.create_string_buffer(str(label).encode())   # kept alive with the trace
        fn = ctypes.cast(LIB.peps_progress_stderr, ctypes.c_void_p)
        _raise(LIB.peps_trace_set_progress(self.h, fn, ctypes.cast(self._label, ctypes.c_void_p)),
               "peps_trace_set_progress")

    def close(self):
        if self.h:
            LIB.peps_trace_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown: the library may already be gone
            pass


def _tr(trace):
    return ctypes.c_void_p(trace.h) if trace is not None else None


def new_status(device):
    return torch.zeros(1, dtype=torch.int32, device=device)


def check(status, where="device"):
    code = int(status.item())
    if code != 0 and code != 1:
        raise PepsError(code, where)
    return code


def peps_eval_batch(desc: Desc, theta, configs, want_e=True, status=None, trace=None):
    """(log_abs [n] f64, sign [n] i8, e_loc [n] f64 or None, status)."""
    theta = _theta(desc, theta)
    configs = _configs(desc, configs)
    _check_dev(theta, configs)
    n = configs.shape[0]
    dev = theta.device
    log_abs = torch.empty(n, dtype=torch.float64, device=dev)
    sign = torch.empty(n, dtype=torch.int8, device=dev)
    e_loc = torch.empty(n, dtype=torch.float64, device=dev) if want_e else None
    status = new_status(dev) if status is None else status
    ws = _chain_ws(desc, n, _lib.WS_EVAL, dev)
    code = LIB.peps_eval_batch(ctypes.byref(desc.c()), _ptr(theta), n, _ptr(configs), _ptr(log_abs), _ptr(sign),
                               _ptr(e_loc), _ptr(status), _ptr(ws), ws.numel(), _tr(trace), _stream())
    _raise(code, "peps_eval_batch")
    return log_abs, sign, e_loc, status


def peps_grad_batch(desc: Desc, theta, configs, status=None, trace=None):
    """(O_rows [n, nnz] f64, log_abs [n] f64, status)."""
    theta = _theta(desc, theta)
    configs = _configs(desc, configs)
    _check_dev(theta, configs)
    n = configs.shape[0]
    dev = theta.device
    O = torch.empty((n, peps_orow_count(desc)), dtype=torch.float64, device=dev)
    log_abs = torch.empty(n, dtype=torch.float64, device=dev)
    status = new_status(dev) if status is None else status
    ws = _chain_ws(desc, n, _lib.WS_GRAD, dev)
    code = LIB.peps_grad_batch(ctypes.byref(desc.c()), _ptr(theta), n, _ptr(configs), _ptr(O), _ptr(log_abs),
                               _ptr(status), _ptr(ws), ws.numel(), _tr(trace), _stream())
    _raise(code, "peps_grad_batch")
    return O, log_abs, status


def peps_sample_sweep(desc: Desc, theta, configs, seed, sweep0, n_sweeps, measure=True, want_O=True,
                      n_accept=None, status=None, out=None, sweep_counter=None, ws=None, want_configs=False,
                      trace=None):
    """Runs n_sweeps sweeps in place on `configs`.  Returns a dict with
    log_abs / sign / e_loc [n_sweeps, n] and O [n_sweeps, n, nnz] (when
    measured), configs [n_sweeps, n, N] (the configuration of every
    measurement, when want_configs), n_accept [n, 3] and status.  `out` may
    supply preallocated output tensors with those keys (checked for shape,
    dtype and contiguity).  `sweep_counter` (int64 [1] on the device,
    optional) is added to sweep0 on the device and advanced by n_sweeps,
    which makes the call replayable from a captured graph.  `ws` (uint8
    device tensor of at least workspace_bytes(desc, n, "sweep") bytes,
    optional) replaces the shared workspace cache; a captured call should
    own its workspace so that no later call can reallocate it."""
    theta = _theta(desc, theta)
    configs = _configs(desc, configs)
    _check_dev(theta, configs)
    n = configs.shape[0]
    dev = theta.device
    res = {} if out is None else dict(out)
    shapes = {"log_abs": ((n_sweeps, n), torch.float64), "sign": ((n_sweeps, n), torch.int8),
              "e_loc": ((n_sweeps, n), torch.float64),
              "O": ((n_sweeps, n, peps_orow_count(desc)), torch.float64),
              "configs": ((n_sweeps, n, desc.N), torch.uint8)}
    if measure:
        for k in ("log_abs", "sign", "e_loc"):
            res.setdefault(k, torch.empty(shapes[k][0], dtype=shapes[k][1], device=dev))
        if want_O:
            res.setdefault("O", torch.empty(shapes["O"][0], dtype=torch.float64, device=dev))
        if want_configs:
            res.setdefault("configs", torch.empty(shapes["configs"][0], dtype=torch.uint8, device=dev))
    for k, t in res.items():
        if k in shapes and t is not None:
            if tuple(t.shape) != shapes[k][0] or t.dtype != shapes[k][1] or not t.is_contiguous() or t.device != dev:
                raise ValueError("out[%r] must be a contiguous %s device tensor of shape %s"
                                 % (k, shapes[k][1], shapes[k][0]))
    if n_accept is None:
        n_accept = torch.zeros((n, 3), dtype=torch.int32, device=dev)
    elif n_accept.dtype != torch.int32 or tuple(n_accept.shape) != (n, 3) or not n_accept.is_contiguous():
        raise ValueError("n_accept must be a contiguous int32 [n, 3] device tensor")
    status = new_status(dev) if status is None else status
    if sweep_counter is not None:
        _check_dev(sweep_counter)
        if sweep_counter.dtype != torch.int64 or sweep_counter.numel() != 1:
            raise ValueError("sweep_counter must be a one-element int64 device tensor")
    ws = _chain_ws(desc, n, _lib.WS_SWEEP, dev, ws)
    code = LIB.peps_sample_sweep(ctypes.byref(desc.c()), _ptr(theta), n, _ptr(configs), int(seed), int(sweep0),
                                 _ptr(sweep_counter), int(n_sweeps), _ptr(res.get("log_abs")), _ptr(res.get("sign")),
                                 _ptr(res.get("e_loc")), _ptr(res.get("O")), _ptr(res.get("configs")),
                                 _ptr(n_accept), _ptr(status), _ptr(ws), ws.numel(), _tr(trace), _stream())
    _raise(code, "peps_sample_sweep")
    res["n_accept"] = n_accept
    res["status"] = status
    return res


def sr_cg_solve(desc: Desc, configs, O_rows, e_loc, tau, eps, max_iter, rtol, weights=None, want_g=True,
                theta=None, status=None, ws=None, log_abs=None, trace=None):
    """(dtheta [N_p], g [N_p] or None, stats [5] = (Ebar, |r|, iters, |b|,
    not-converged flag), status).  Averages are weighted by `weights` [n_s]
    when given, else by |rho|^(2 - alpha) formed on the device from
    `log_abs` [n_s] when given (Eq. A1), else uniform.  When `theta`
    (float64 [N_p], device) is given it is updated in place: theta +=
    dtheta.  `ws`: optional caller-owned workspace of at least
    workspace_bytes(desc, n_s, "sr") bytes."""
    configs = _configs(desc, configs)
    n_s = configs.shape[0]
    if O_rows.dtype != torch.float64 or O_rows.shape != (n_s, peps_orow_count(desc)) or not O_rows.is_contiguous():
        raise ValueError("O_rows must be contiguous float64 [n_s, nnz]")
    if e_loc.dtype != torch.float64 or e_loc.shape != (n_s,):
        raise ValueError("e_loc must be float64 [n_s]")
    for name, v in (("weights", weights), ("log_abs", log_abs)):
        if v is not None and (v.dtype != torch.float64 or v.shape != (n_s,) or not v.is_contiguous()):
            raise ValueError("%s must be a contiguous float64 [n_s] tensor" % name)
    _check_dev(configs, O_rows, e_loc, weights, theta, log_abs)
    dev = O_rows.device
    n_p = peps_param_count(desc)
    if theta is not None and (theta.dtype != torch.float64 or theta.shape != (n_p,) or not theta.is_contiguous()):
        raise ValueError("theta must be a contiguous float64 vector of length N_p")
    dtheta = torch.empty(n_p, dtype=torch.float64, device=dev)
    g = torch.empty(n_p, dtype=torch.float64, device=dev) if want_g else None
    stats = torch.zeros(_lib.SR_NSTATS, dtype=torch.float64, device=dev)
    status = new_status(dev) if status is None else status
    ws = _own_ws(ws, "sr", peps_workspace_bytes(desc, n_s, _lib.WS_SR), dev)
    code = LIB.sr_cg_solve(ctypes.byref(desc.c()), n_s, _ptr(configs), _ptr(O_rows), _ptr(weights), _ptr(log_abs),
                           _ptr(e_loc.contiguous()), float(tau), float(eps), int(max_iter), float(rtol),
                           _ptr(dtheta), _ptr(g), _ptr(theta), _ptr(stats), _ptr(status), _ptr(ws), ws.numel(),
                           _tr(trace), _stream())
    _raise(code, "sr_cg_solve")
    return dtheta, g, stats, status


def sr_cg_solve_noalloc(desc: Desc, configs, O_rows, e_loc, tau, eps, max_iter, rtol, weights=None, want_g=True,
                        theta=None, status=None, log_abs=None, out=None):
    """sr_cg_solve for callers that cannot allocate device memory: the
    library's fixed per-GPU scratch replaces the workspace.  `out` may
    supply the output tensors dtheta [N_p], g [N_p] (or None) and stats [5]
    as a dict, so that the call itself allocates nothing; otherwise they are
    allocated here before the call.  Returns (dtheta, g, stats, status)."""
    configs = _configs(desc, configs)
    n_s = configs.shape[0]
    if O_rows.dtype != torch.float64 or O_rows.shape != (n_s, peps_orow_count(desc)) or not O_rows.is_contiguous():
        raise ValueError("O_rows must be contiguous float64 [n_s, nnz]")
    if e_loc.dtype != torch.float64 or e_loc.shape != (n_s,) or not e_loc.is_contiguous():
        raise ValueError("e_loc must be contiguous float64 [n_s]")
    for name, v in (("weights", weights), ("log_abs", log_abs)):
        if v is not None and (v.dtype != torch.float64 or v.shape != (n_s,) or not v.is_contiguous()):
            raise ValueError("%s must be a contiguous float64 [n_s] tensor" % name)
    _check_dev(configs, O_rows, e_loc, weights, theta, log_abs)
    dev = O_rows.device
    n_p = peps_param_count(desc)
    if theta is not None and (theta.dtype != torch.float64 or theta.shape != (n_p,) or not theta.is_contiguous()):
        raise ValueError("theta must be a contiguous float64 vector of length N_p")
    out = {} if out is None else out
    dtheta = out.get("dtheta")
    if dtheta is None:
        dtheta = torch.empty(n_p, dtype=torch.float64, device=dev)
    g = out.get("g", None if not want_g else torch.empty(n_p, dtype=torch.float64, device=dev))
    stats = out.get("stats")
    if stats is None:
        stats = torch.zeros(_lib.SR_NSTATS, dtype=torch.float64, device=dev)
    for t, shape in ((dtheta, (n_p,)), (g, (n_p,)), (stats, (_lib.SR_NSTATS,))):
        if t is not None and (t.dtype != torch.float64 or tuple(t.shape) != shape or not t.is_contiguous()
                              or t.device != dev):
            raise ValueError("outputs must be contiguous float64 device tensors of the documented shapes")
    status = new_status(dev) if status is None else status
    code = LIB.sr_cg_solve_noalloc(ctypes.byref(desc.c()), n_s, _ptr(configs), _ptr(O_rows), _ptr(weights),
                                   _ptr(log_abs), _ptr(e_loc), float(tau), float(eps), int(max_iter), float(rtol),
                                   _ptr(dtheta), _ptr(g), _ptr(theta), _ptr(stats), _ptr(status), _stream())
    _raise(code, "sr_cg_solve_noalloc")
    return dtheta, g, stats, status


def peps_sample_stats(desc: Desc, values, n_chains, log_abs=None, weights=None):
    """Weighted means and standard errors of per-sample quantities:
    values [n_sweeps * n_chains, k] (or [n_sweeps * n_chains]) float64 in
    the sample order of peps_sample_sweep; weights `weights` when given,
    else |rho|^(2 - alpha) from `log_abs` when given, else uniform.  Returns
    a device tensor [k, 2] (mean, standard error of the mean from the
    per-chain means)."""
    v = values if values.dim() == 2 else values.reshape(-1, 1)
    if v.dtype != torch.float64 or not v.is_contiguous():
        raise ValueError("values must be contiguous float64")
    n_s, k = v.shape
    if n_chains < 1 or n_s % n_chains != 0:
        raise ValueError("the sample count must be a multiple of n_chains")
    for name, x in (("log_abs", log_abs), ("weights", weights)):
        if x is not None and (x.dtype != torch.float64 or x.numel() != n_s or not x.is_contiguous()):
            raise ValueError("%s must be contiguous float64 with one entry per sample" % name)
    _check_dev(v, log_abs, weights)
    out = torch.empty((k, 2), dtype=torch.float64, device=v.device)
    _raise(LIB.peps_sample_stats(ctypes.byref(desc.c()), n_s // n_chains, int(n_chains), k, _ptr(v), _ptr(weights),
                                 _ptr(log_abs), _ptr(out), _stream()), "peps_sample_stats")
    return out


def peps_autotune_compression(desc: Desc, theta, configs, repeats=2, status=None):
    """Times the boundary compression of these configurations with every
    compression kernel valid for desc's shape (a host call: synchronises).
    Returns (best kernel, {kernel name: ms per full boundary pass})."""
    theta = _theta(desc, theta)
    configs = _configs(desc, configs)
    _check_dev(theta, configs)
    n = configs.shape[0]
    dev = theta.device
    need = 0
    for k in (_lib.COMPRESS_REGISTER, _lib.COMPRESS_LDS, _lib.COMPRESS_WORKSPACE):
        try:
            need = max(need, peps_workspace_bytes(dataclasses.replace(desc, compress_kernel=k), n, _lib.WS_EVAL))
        except PepsError:
            pass
    ws = _ws("chain", need, dev)
    status = new_status(dev) if status is None else status
    ms = (ctypes.c_double * 4)()
    best = ctypes.c_int32(0)
    code = LIB.peps_autotune_compression(ctypes.byref(desc.c()), _ptr(theta), n, _ptr(configs), int(repeats), ms,
                                         ctypes.byref(best), _ptr(status), _ptr(ws), ws.numel(), _stream())
    _raise(code, "peps_autotune_compression")
    check(status, "peps_autotune_compression")
    return int(best.value), {_lib.COMPRESS_NAMES[k]: ms[k] for k in (1, 2, 3) if ms[k] >= 0.0}


def peps_direct_workspace_bytes(desc: Desc, n_chains, chi_dl) -> int:
    out = ctypes.c_size_t(0)
    _raise(LIB.peps_direct_workspace_bytes(ctypes.byref(desc.c()), int(n_chains), int(chi_dl), ctypes.byref(out)),
           "peps_direct_workspace_bytes")
    return int(out.value)


def peps_direct_sample(desc: Desc, theta, n_chains, chi_dl, seed, draw=0, reweight=False, b_diag=None,
                       update_b=False, reuse_double_layer=False, status=None, out=None, ws=None, trace=None):
    """Direct (autoregressive) draws, one configuration per chain.  Returns
    (configs [n, N] u8, log_p [n] f64, status).  `b_diag` (float64 [1] on the
    device) is read when reweight and updated in place when update_b.  `out`
    may supply (configs, log_p) tensors; `ws` a uint8 workspace of at least
    peps_direct_workspace_bytes(desc, n_chains, chi_dl) bytes.  With
    reuse_double_layer the double layer of the previous call on the same
    workspace is reused (theta unchanged since; needs an explicit `ws`)."""
    if reuse_double_layer and ws is None:
        raise ValueError("reuse_double_layer needs the workspace of the previous call (ws=)")
    theta = _theta(desc, theta)
    _check_dev(theta, b_diag)
    dev = theta.device
    n = int(n_chains)
    if (reweight or update_b) and (b_diag is None or b_diag.dtype != torch.float64 or b_diag.numel() != 1):
        raise ValueError("b_diag must be a float64 device tensor with one element")
    if out is None:
        configs = torch.empty((n, desc.N), dtype=torch.uint8, device=dev)
        log_p = torch.empty(n, dtype=torch.float64, device=dev)
    else:
        configs, log_p = out
        if (configs.dtype != torch.uint8 or tuple(configs.shape) != (n, desc.N) or not configs.is_contiguous()
                or log_p.dtype != torch.float64 or log_p.numel() != n or not log_p.is_contiguous()):
            raise ValueError("out must be (uint8 [n, N], float64 [n]) contiguous tensors")
    status = new_status(dev) if status is None else status
    need = peps_direct_workspace_bytes(desc, n, chi_dl)
    ws = _own_ws(ws, "direct", need, dev)
    code = LIB.peps_direct_sample(ctypes.byref(desc.c()), _ptr(theta), n, int(chi_dl), int(seed), int(draw),
                                  int(bool(reweight)), _ptr(b_diag), int(bool(update_b)),
                                  int(bool(reuse_double_layer)), _ptr(configs), _ptr(log_p),
                                  _ptr(status), _ptr(ws), ws.numel(), _tr(trace), _stream())
    _raise(code, "peps_direct_sample")
    return configs, log_p, status


def peps_importance_weights(log_abs, log_p, out=None):
    """Eq. A7 weights |rho|^2 / p of directly drawn samples, largest = 1."""
    for x in (log_abs, log_p):
        if x.dtype != torch.float64 or not x.is_contiguous() or x.dim() != 1:
            raise ValueError("log_abs and log_p must be contiguous float64 vectors")
    if log_abs.numel() != log_p.numel() or log_abs.numel() < 1:
        raise ValueError("log_abs and log_p must have the same nonzero length")
    _check_dev(log_abs, log_p)
    w = torch.empty_like(log_abs) if out is None else out
    _raise(LIB.peps_importance_weights(log_abs.numel(), _ptr(log_abs), _ptr(log_p), _ptr(w), _stream()),
           "peps_importance_weights")
    return w


def peps_vjp_batch(desc: Desc, configs, O_rows, cot):
    """grad [N_p] f64 = sum_i cot_i O_i, scattered into the parameter layout."""
    configs = _configs(desc, configs)
    n = configs.shape[0]
    if O_rows.dtype != torch.float64 or O_rows.shape != (n, peps_orow_count(desc)) or not O_rows.is_contiguous():
        raise ValueError("O_rows must be contiguous float64 [n, nnz]")
    if cot.dtype != torch.float64 or cot.shape != (n,):
        raise ValueError("cot must be float64 [n]")
    _check_dev(configs, O_rows, cot)
    grad = torch.empty(peps_param_count(desc), dtype=torch.float64, device=O_rows.device)
    ws = _ws("sr", peps_workspace_bytes(desc, n, _lib.WS_SR), O_rows.device)
    code = LIB.peps_vjp_batch(ctypes.byref(desc.c()), n, _ptr(configs), _ptr(O_rows), _ptr(cot.contiguous()),
                              _ptr(grad), _ptr(ws), ws.numel(), _stream())
    _raise(code, "peps_vjp_batch")
    return grad


OBS_NAMES = ("mz", "mz2", "n", "docc")


def peps_observables_batch(desc: Desc, configs):
    """Local values [n, 4] f64 of M_z, M_z^2, particle number and double
    occupancy, (A(s) + A(s')) / 2 per sample (columns in OBS_NAMES order)."""
    configs = _configs(desc, configs)
    _check_dev(configs)
    n = configs.shape[0]
    out = torch.empty((n, _lib.N_OBS), dtype=torch.float64, device=configs.device)
    _raise(LIB.peps_observables_batch(ctypes.byref(desc.c()), n, _ptr(configs), _ptr(out), _stream()),
           "peps_observables_batch")
    return out


def thermal_observables(desc: Desc, configs, beta_phys, n_chains=None, log_abs=None, weights=None):
    """Sample estimates at inverse temperature beta_phys, reduced on the
    device (peps_sample_stats): per-site <M_z^2>/N, the susceptibility
    beta <M_z^2> / N (<M_z>^2 := 0), <n>/N and the double occupancy <D>/N,
    each with its standard error from the per-chain means (n_chains chains,
    samples in sweep-major order; default: one chain per sample), weighted
    by |rho|^(2 - alpha) from `log_abs` when given (Eq. A1).  Host floats;
    synchronises."""
    v = peps_observables_batch(desc, configs)
    n = configs.shape[0]
    st = peps_sample_stats(desc, v, n if n_chains is None else n_chains, log_abs, weights).cpu().numpy()
    N = desc.N
    out = {}
    for q, name in enumerate(("mz_per_site", "mz2_per_site", "n_per_site", "docc_per_site")):
        out[name] = float(st[q, 0]) / N
        out[name + "_stderr"] = float(st[q, 1]) / N
    out["chi"] = beta_phys * out["mz2_per_site"]
    out["chi_stderr"] = beta_phys * out["mz2_per_site_stderr"]
    return out


def su_bond_count(desc: Desc) -> int:
    """Bonds of the lattice: L1 (L2-1) horizontal, then (L1-1) L2 vertical."""
    return desc.L1 * (desc.L2 - 1) + (desc.L1 - 1) * desc.L2


def peps_simple_update(desc: Desc, theta, lambdas, tau, n_steps, status=None, ws=None):
    """n_steps simple-update steps of tau in place on theta (float64 [N_p])
    and the bond weights lambdas (float64 [n_bonds, D], start from ones);
    returns status."""
    if not theta.is_contiguous():
        raise ValueError("theta is updated in place and must be contiguous")
    theta = _theta(desc, theta)
    dev = theta.device
    nb = su_bond_count(desc)
    if lambdas.dtype != torch.float64 or tuple(lambdas.shape) != (nb, desc.D) or not lambdas.is_contiguous():
        raise ValueError("lambdas must be contiguous float64 [n_bonds, D]")
    _check_dev(theta, lambdas)
    status = new_status(dev) if status is None else status
    ws = _own_ws(ws, "su", peps_workspace_bytes(desc, 0, _lib.WS_SU), dev)
    _raise(LIB.peps_simple_update(ctypes.byref(desc.c()), _ptr(theta), _ptr(lambdas), float(tau), int(n_steps),
                                  _ptr(status), _ptr(ws), ws.numel(), _stream()), "peps_simple_update")
    return status


def peps_su_absorb(desc: Desc, theta, lambdas):
    """The plain PEPS of a simple-update state: sqrt(lambda) on both ends of
    every bond (a new tensor)."""
    theta = _theta(desc, theta)
    if lambdas.dtype != torch.float64 or tuple(lambdas.shape) != (su_bond_count(desc), desc.D):
        raise ValueError("lambdas must be float64 [n_bonds, D]")
    _check_dev(theta, lambdas)
    out = torch.empty_like(theta)
    _raise(LIB.peps_su_absorb(ctypes.byref(desc.c()), _ptr(theta), _ptr(lambdas.contiguous()), _ptr(out), _stream()),
           "peps_su_absorb")
    return out


def nnn_spin_correlation(desc: Desc, theta, configs, n_chains=None, log_abs=None, weights=None):
    """F = sum_<<ij>> <S_i.S_j> / M over the M = 2 (L1-1)(L2-1)
    next-nearest-neighbour pairs (Benchmark section, Hubbard model; also
    defined for spins): local energies of the Hamiltonian sum_<<ij>> S_i.S_j
    (J2 = 1, every other coupling 0) from peps_eval_batch, averaged on the
    device (peps_sample_stats; weights `weights`, else |rho|^(2 - alpha)
    from `log_abs`, else uniform) and halved.  Returns (F, its standard error, per-sample local
    values); synchronises."""
    d = dataclasses.replace(desc, J1=0.0, J2=1.0, t=0.0, U=0.0, mu=0.0)
    _, _, e, status = peps_eval_batch(d, theta, configs)
    n = configs.shape[0]
    st = peps_sample_stats(desc, e, n if n_chains is None else n_chains, log_abs, weights)
    check(status, "nnn_spin_correlation")
    m, se = st[0].cpu().tolist()
    M = 2 * (desc.L1 - 1) * (desc.L2 - 1)
    return m / (2.0 * M), se / (2.0 * M), e


def specific_heat(betas, energies, smoothing=None, weights=None):
    """C_v(beta) = -beta^2 dE/dbeta from energies per site on a beta grid,
    through a smoothing cubic spline fitted to E(beta) and differentiated
    (Benchmark section: the specific heat from a spline fit of the energy).
    `smoothing` is the spline's residual budget (scipy's `s`; None
    interpolates), `weights` the inverse standard errors.  Host only; returns
    an array aligned with `betas`."""
    import numpy as np
    from scipy.interpolate import UnivariateSpline
    b = np.asarray(betas, dtype=np.float64)
    e = np.asarray(energies, dtype=np.float64)
    if b.ndim != 1 or b.shape != e.shape or b.size < 5 or np.any(np.diff(b) <= 0):
        raise ValueError("specific_heat: need >= 5 increasing betas and matching energies")
    spl = UnivariateSpline(b, e, w=weights, k=3, s=0.0 if smoothing is None else smoothing)
    return -b * b * spl.derivative()(b)


class PepsLogAmp(torch.autograd.Function):
    """log|psi(S_i)| for a batch of configurations as a differentiable
    function of theta.  Forward: peps_grad_batch (log-amplitudes and the O
    rows of the adjoint contraction, Eq. 8); backward: peps_vjp_batch with
    the incoming cotangent.  Usage: PepsLogAmp.apply(theta, configs, desc)."""

    @staticmethod
    def forward(ctx, theta, configs, desc):
        O, log_abs, status = peps_grad_batch(desc, theta, configs)
        ctx.desc = desc
        ctx.save_for_backward(configs, O, status)
        return log_abs

    @staticmethod
    def backward(ctx, g):
        configs, O, status = ctx.saved_tensors
        check(status, "PepsLogAmp forward")
        grad = peps_vjp_batch(ctx.desc, configs, O, g.to(torch.float64).contiguous())
        return grad, None, None


