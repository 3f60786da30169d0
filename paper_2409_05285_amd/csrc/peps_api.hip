// C ABI of the library: descriptor validation, workspace layout, and the
// launch sequences of the device calls (declared in include/peps.h).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <vector>

#include "peps_chain.hpp"
#include "peps_common.hpp"
#include "peps_kernels.hpp"

using namespace peps;

// Caller-owned instrumentation record (declared opaque in peps.h).
struct peps_trace {
  int capacity = 0, used = 0;
  std::vector<hipEvent_t> a, b;
  std::vector<int> cls;
  // progress hook: one payload per launch slot (stable addresses)
  struct Note {
    peps_progress_fn fn;
    void* user;
    int32_t cls, launch;
  };
  peps_progress_fn fn = nullptr;
  void* user = nullptr;
  std::vector<Note> notes;
};

namespace {


bool desc_ok(const peps_desc* d) {
  if (!d) return false;
  if (d->L1 < 2 || d->L2 < 2 || d->L1 > MAX_L || d->L2 > MAX_L || d->L1 * d->L2 > MAX_SITES) return false;
  if (d->D < 1 || d->chi < 1) return false;
  if (d->model == PEPS_MODEL_HEISENBERG) {
    if (d->d != 2) return false;
  } else if (d->model == PEPS_MODEL_HUBBARD) {
    if (d->d != 4) return false;
  } else {
    return false;
  }
  if (d->alpha != 1 && d->alpha != 2) return false;
  if (d->fermionic != 0 && d->fermionic != 1) return false;
  if (d->fermionic && d->model != PEPS_MODEL_HUBBARD) return false;
  if (d->precision != PEPS_PREC_FP64 && d->precision != PEPS_PREC_MIXED) return false;
  if (d->compress_kernel < PEPS_COMPRESS_AUTO || d->compress_kernel > PEPS_COMPRESS_WORKSPACE) return false;
  if (!isfinite(d->J1) || !isfinite(d->J2) || !isfinite(d->t) || !isfinite(d->U) || !isfinite(d->mu)) return false;
  return true;
}

// Problem and per-chain workspace layout.  refl_store selects, for the
// workspace-resident compression, the layout that keeps every site's QR
// reflectors (faster) or the one that keeps only the R factors and rebuilds
// the reflectors (smaller).
Prob make_prob(const peps_desc* d, bool refl_store = true) {
  Prob P;
  memset(&P, 0, sizeof(P));
  P.L1 = d->L1;
  P.L2 = d->L2;
  P.N = d->L1 * d->L2;
  P.d = d->d;
  P.d2 = d->d * d->d;
  P.D = d->D;
  P.chi = d->chi;
  P.model = d->model;
  P.alpha = d->alpha;
  P.fermionic = d->fermionic;
  P.nb_moves = d->model == PEPS_MODEL_HEISENBERG ? 2 : 4;
  P.ns_moves = d->model == PEPS_MODEL_HEISENBERG ? 1 : 2;
  P.n_slots = P.L1 * (P.nb_moves * (P.L2 - 1) + P.ns_moves * P.L2) + (P.L1 - 1) * P.nb_moves * P.L2;
  P.J1 = d->J1;
  P.J2 = d->J2;
  P.t = d->t;
  P.U = d->U;
  P.mu = d->mu;
  int64_t np = 0, nnz = 0;
  for (int r = 0; r < P.L1; ++r)
    for (int c = 0; c < P.L2; ++c) {
      int bs = block_size(P, r, c);
      nnz += bs;
      np += (int64_t)P.d2 * bs;
    }
  P.nnz = nnz;
  P.np = np;
  const int64_t cd = (int64_t)P.chi * P.D;
  P.TS = (int)(P.chi * P.D * P.chi);
  P.BS = (int)(cd * P.D * cd);
  P.ES = (int)(P.chi * P.D * P.D * P.chi);
  P.XS = (int)(P.chi * P.chi * P.D * P.D * P.D);
  auto pad = [](int64_t x) { return (x + 31) & ~(int64_t)31; };
  int64_t off = 0;
  P.off_top = off;   off += pad((int64_t)P.L1 * P.L2 * P.TS);
  P.off_lstop = off; off += pad(P.L1);
  P.off_bot = off;   off += pad((int64_t)P.L1 * P.L2 * P.TS);
  P.off_lsbot = off; off += pad(P.L1);
  // the workspace-resident compression keeps one QR matrix and the R factor
  // of every site (it rebuilds a site's reflectors when it needs them); the
  // other kernels keep every site's absorbed tensor or reflectors
  P.ckernel = d->compress_kernel != PEPS_COMPRESS_AUTO
                  ? d->compress_kernel
                  : (compress2_supported(P) ? PEPS_COMPRESS_REGISTER
                                            : (compress_in_lds(P) ? PEPS_COMPRESS_LDS : PEPS_COMPRESS_WORKSPACE));
  P.cauto = d->compress_kernel == PEPS_COMPRESS_AUTO;
  const bool big = P.ckernel == PEPS_COMPRESS_WORKSPACE;
  const bool rebuild = big && !refl_store;
  P.refl_store = rebuild ? 0 : 1;
  P.off_B = off;     off += pad(rebuild ? (int64_t)P.BS : (int64_t)P.L2 * P.BS);
  P.off_Rst = off;   if (rebuild) off += pad((int64_t)P.L2 * cd * cd);
  P.off_tmp = off;   off += pad(P.BS);
  P.off_R = off;     off += pad((int64_t)(P.L2 + 1) * P.ES);
  P.off_L = off;     off += pad(4 * (int64_t)P.ES);
  {
    // strip intermediates; also the general compression kernel's work
    // matrices when they exceed its LDS
    const int64_t xs = 2 * (int64_t)P.XS, cs = (int64_t)(compress_dyn_lds(P) / sizeof(double));
    P.off_X = off;   off += pad(xs > cs ? xs : cs);
  }
  P.off_epart = off; off += pad(epart_size(P));
  P.off_tau = off;   off += pad((int64_t)P.L2 * P.chi * P.D);
  P.off_T = off;
  if (big) off += pad((int64_t)compress_big_T_doubles(P));
  P.mixed = d->precision == PEPS_PREC_MIXED;
  if (P.mixed) {
    // FP32 copies of the boundaries, same element strides as the FP64 ones
    const int64_t nf = (int64_t)P.L1 * P.L2 * P.TS;
    P.off_top32 = off; off += pad((nf + 1) / 2);
    P.off_bot32 = off; off += pad((nf + 1) / 2);
  }
  P.chain_stride = off;
  return P;
}

// Checks that the compiled tile limits hold for the device path.
peps_status device_support(const peps_desc* d, const Prob& P) {
  (void)d;
  if ((int64_t)P.chi * P.D > CD_MAX) return PEPS_ERR_UNSUPPORTED;   // compression column arrays
  if (P.chi > 255) return PEPS_ERR_UNSUPPORTED;                    // compressed bond table (8 bits)
  if (P.ckernel == PEPS_COMPRESS_REGISTER && !compress2_supported(P)) return PEPS_ERR_UNSUPPORTED;
  if (P.ckernel == PEPS_COMPRESS_LDS && !compress_in_lds(P)) return PEPS_ERR_UNSUPPORTED;
  return PEPS_OK;
}

#define HIP_TRY(x)                          \
  do {                                      \
    if ((x) != hipSuccess) return PEPS_ERR_HIP; \
  } while (0)

// Instrumentation: a launch bracketed by two events of the caller's trace.
struct TraceScope {
  peps_trace* t;
  int idx = -1;
  hipStream_t st;
  TraceScope(peps_trace* t_, int cls, hipStream_t s) : t(t_), st(s) {
    if (!t || t->used >= t->capacity) return;
    idx = t->used++;
    t->cls[idx] = cls;
    (void)hipEventRecord(t->a[idx], st);
  }
  ~TraceScope() {
    if (idx < 0) return;
    (void)hipEventRecord(t->b[idx], st);
    if (t->fn) {
      peps_trace::Note& n = t->notes[idx];
      n.fn = t->fn;
      n.user = t->user;
      n.cls = t->cls[idx];
      n.launch = idx;
      (void)hipLaunchHostFunc(st, &TraceScope::notify, &n);
    }
  }
  static void notify(void* p) {
    const peps_trace::Note* n = (const peps_trace::Note*)p;
    n->fn(n->user, n->cls, n->launch);
  }
};

// Row compression by the kernel the problem selected (make_prob).  Chosen
// automatically, the register-resident kernel gives way to the LDS-resident
// one (same workspace layout) for batches of 512 chains or more when
// chi D^2 <= 64: its 256-thread workgroups fit more chains per CU, which
// measured 1.1-2.9 times faster there, while with fewer chains, or larger
// matrices, the register kernel was as fast or faster.
hipError_t compress_row(const Prob& P, int n, int dir, int r, const double* theta, const uint8_t* configs,
                        double* ws, int32_t* status, hipStream_t st) {
  int k = P.ckernel;
  if (P.cauto && k == PEPS_COMPRESS_REGISTER && n >= 512 && (int64_t)P.chi * P.D * P.D <= 64 && compress_in_lds(P))
    k = PEPS_COMPRESS_LDS;
  if (k == PEPS_COMPRESS_REGISTER) return launch_compress2(P, n, dir, r, theta, configs, ws, status, st);
  if (k == PEPS_COMPRESS_LDS) return launch_compress(P, n, dir, r, theta, configs, ws, status, st);
  return launch_compress_big(P, n, dir, r, theta, configs, ws, status, st);
}

// Mixed precision: the FP32 copy of theta, placed after the chain
// workspaces, then the list of row strips to measure again in FP64 (count
// and up to 2 L1 - 1 items per chain).
size_t theta32_bytes(const Prob& P) { return P.mixed ? (size_t)((P.np + 63) & ~(int64_t)63) * sizeof(float) : 0; }
float* theta32_ptr(const Prob& P, double* ws, int64_t n) {
  return P.mixed ? (float*)(ws + (size_t)n * P.chain_stride) : nullptr;
}
size_t redo_list_bytes(const Prob& P, int64_t n) {
  // count, then up to 2 L1 - 1 row strips per chain
  return P.mixed ? (size_t)((n * (2 * P.L1 - 1) + 1) * sizeof(int32_t) + 255) & ~(size_t)255 : 0;
}
int32_t* redo_list_ptr(const Prob& P, double* ws, int64_t n) {
  return P.mixed ? (int32_t*)((char*)(ws + (size_t)n * P.chain_stride) + theta32_bytes(P)) : nullptr;
}

#define TIMED(cls, call)            \
  do {                              \
    TraceScope _ts(trace, (cls), st); \
    HIP_TRY(call);                  \
  } while (0)

}  // namespace

extern "C" {

int64_t peps_param_count(const peps_desc* d) {
  if (!desc_ok(d)) return -1;
  return make_prob(d).np;
}

int64_t peps_orow_count(const peps_desc* d) {
  if (!desc_ok(d)) return -1;
  return make_prob(d).nnz;
}

int64_t peps_slot_count(const peps_desc* d) {
  if (!desc_ok(d)) return -1;
  return make_prob(d).n_slots;
}

static size_t chain_ws_bytes(const Prob& P, int64_t n) {
  return (size_t)n * (size_t)P.chain_stride * sizeof(double) + theta32_bytes(P) + redo_list_bytes(P, n);
}

peps_status peps_workspace_bytes(const peps_desc* d, int64_t n, int32_t what, size_t* bytes) {
  if (!desc_ok(d) || !bytes || n < 0) return PEPS_ERR_ARG;
  Prob P = make_prob(d);
  switch (what) {
    case PEPS_WS_EVAL:
    case PEPS_WS_GRAD:
    case PEPS_WS_SWEEP:
      *bytes = chain_ws_bytes(P, n);
      return PEPS_OK;
    case PEPS_WS_MIN:
      *bytes = chain_ws_bytes(make_prob(d, false), n);
      return PEPS_OK;
    case PEPS_WS_SU:
      *bytes = (size_t)su_max_group(P) * ((su_bond_doubles(P) + 31) & ~(size_t)31) * sizeof(double);
      return PEPS_OK;
    case PEPS_WS_SR:
      *bytes = sr_workspace_bytes(P, n);
      return PEPS_OK;
    default:
      return PEPS_ERR_ARG;
  }
}

const char* peps_status_string(peps_status s) {
  switch (s) {
    case PEPS_OK: return "ok";
    case PEPS_ERR_ARG: return "invalid argument or shape";
    case PEPS_ERR_UNSUPPORTED: return "valid but beyond the compiled tile limits of the device path";
    case PEPS_ERR_HIP: return "HIP runtime or launch failure";
    case PEPS_ERR_WORKSPACE: return "workspace smaller than peps_workspace_bytes()";
    case PEPS_ERR_NONFINITE: return "non-finite value in the data";
    case PEPS_ERR_ZERO_AMPLITUDE: return "zero strip amplitude for a sample";
    case PEPS_ERR_CG_BREAKDOWN: return "conjugate gradient breakdown (p^T A p <= 0)";
    case PEPS_WARN_CG_NOT_CONVERGED: return "conjugate gradient reached max_iter";
    default: return "unknown status";
  }
}

static peps_status common_checks(const peps_desc* d, Prob& P, int64_t n, const void* theta, const void* configs,
                                 void* ws, size_t ws_bytes, int what) {
  if (!desc_ok(d)) return PEPS_ERR_ARG;
  if (n < 0 || n > (1 << 24)) return PEPS_ERR_ARG;
  P = make_prob(d);
  peps_status s = device_support(d, P);
  if (s != PEPS_OK) return s;
  if (n == 0) return PEPS_OK;
  if (!configs || !ws || (what != PEPS_WS_SR && !theta)) return PEPS_ERR_ARG;
  // the full layout when the workspace holds it, else the smaller one
  if (ws_bytes < chain_ws_bytes(P, n)) {
    P = make_prob(d, false);
    if (ws_bytes < chain_ws_bytes(P, n)) return PEPS_ERR_WORKSPACE;
  }
  return PEPS_OK;
}

static peps_status compress_all_bots(const Prob& P, int n, const double* theta, const uint8_t* configs, double* ws,
                                     int32_t* status, peps_trace* trace, hipStream_t st) {
  for (int r = P.L1 - 1; r >= 1; --r) TIMED(PEPS_K_COMPRESS, compress_row(P, n, 1, r, theta, configs, ws, status, st));
  return PEPS_OK;
}

// Measurement of every chain's configuration from its top and bottom
// boundaries.  Mixed precision: the FP32 pass estimates each sample's
// rounding error; the samples above the bar are listed and measured again
// by one persistent FP64 launch over their row strips, and their outputs
// rewritten.
static peps_status measure(const Prob& P, int n, const double* theta, const float* t32, const uint8_t* configs,
                           double* ws, double* log_abs, int8_t* sign, double* e_loc, double* O_rows, int64_t out_off,
                           int32_t* status, peps_trace* trace, hipStream_t st) {
  const int want_e = e_loc != nullptr;
  for (int r = 0; r < P.L1; ++r)
    TIMED(PEPS_K_MEAS1, launch_meas1(P, n, r, theta, t32, configs, ws, O_rows, want_e, status, st));
  if (want_e)
    for (int r = 0; r < P.L1 - 1; ++r) TIMED(PEPS_K_MEAS2, launch_meas2(P, n, r, theta, t32, configs, ws, status, st));
  TIMED(PEPS_K_FINAL, launch_finalize(P, n, configs, ws, log_abs, sign, e_loc, out_off, want_e, 0, status, st));
  if (P.mixed) {
    int32_t* list = redo_list_ptr(P, ws, n);
    TIMED(PEPS_K_FINAL, launch_redo_flags(P, n, ws, want_e, list, st));
    TIMED(PEPS_K_FINAL, launch_remeasure(P, n, theta, configs, ws, list, O_rows, want_e, status, st));
    TIMED(PEPS_K_FINAL, launch_finalize(P, n, configs, ws, log_abs, sign, e_loc, out_off, want_e, 1, status, st));
  }
  return PEPS_OK;
}

peps_status peps_eval_batch(const peps_desc* d, const double* theta, int32_t n, const uint8_t* configs,
                            double* log_abs, int8_t* sign, double* e_loc, int32_t* status, void* ws,
                            size_t ws_bytes, peps_trace* trace, peps_stream_t stream) {
  Prob P;
  peps_status s = common_checks(d, P, n, theta, configs, ws, ws_bytes, PEPS_WS_EVAL);
  if (s != PEPS_OK || n == 0) return s;
  if (!log_abs || !sign) return PEPS_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  double* w = (double*)ws;
  float* t32 = theta32_ptr(P, w, n);
  HIP_TRY(launch_check_digits(P, n, configs, status, st));
  if (t32) HIP_TRY(launch_theta32(P, theta, t32, st));
  for (int r = 0; r <= P.L1 - 2; ++r) TIMED(PEPS_K_COMPRESS, compress_row(P, n, 0, r, theta, configs, w, status, st));
  s = compress_all_bots(P, n, theta, configs, w, status, trace, st);
  if (s != PEPS_OK) return s;
  return measure(P, n, theta, t32, configs, w, log_abs, sign, e_loc, nullptr, 0, status, trace, st);
}

peps_status peps_grad_batch(const peps_desc* d, const double* theta, int32_t n, const uint8_t* configs,
                            double* O_rows, double* log_abs, int32_t* status, void* ws, size_t ws_bytes,
                            peps_trace* trace, peps_stream_t stream) {
  Prob P;
  peps_status s = common_checks(d, P, n, theta, configs, ws, ws_bytes, PEPS_WS_GRAD);
  if (s != PEPS_OK || n == 0) return s;
  if (!O_rows) return PEPS_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  double* w = (double*)ws;
  float* t32 = theta32_ptr(P, w, n);
  HIP_TRY(launch_check_digits(P, n, configs, status, st));
  if (t32) HIP_TRY(launch_theta32(P, theta, t32, st));
  for (int r = 0; r <= P.L1 - 2; ++r) TIMED(PEPS_K_COMPRESS, compress_row(P, n, 0, r, theta, configs, w, status, st));
  s = compress_all_bots(P, n, theta, configs, w, status, trace, st);
  if (s != PEPS_OK) return s;
  return measure(P, n, theta, t32, configs, w, log_abs, nullptr, nullptr, O_rows, 0, status, trace, st);
}

peps_status peps_sample_sweep(const peps_desc* d, const double* theta, int32_t n_chains, uint8_t* configs,
                              uint64_t seed, uint64_t sweep0, uint64_t* sweep_counter, int32_t n_sweeps,
                              double* log_abs, int8_t* sign, double* e_loc, double* O_rows,
                              uint8_t* sample_configs, int32_t* n_accept, int32_t* status, void* ws,
                              size_t ws_bytes, peps_trace* trace, peps_stream_t stream) {
  Prob P;
  peps_status s = common_checks(d, P, n_chains, theta, configs, ws, ws_bytes, PEPS_WS_SWEEP);
  if (s != PEPS_OK || n_chains == 0) return s;
  if (n_sweeps < 0) return PEPS_ERR_ARG;
  const bool measure_any = log_abs || sign || e_loc || O_rows || sample_configs;
  hipStream_t st = (hipStream_t)stream;
  double* w = (double*)ws;
  const int n = n_chains;
  float* t32 = theta32_ptr(P, w, n);
  HIP_TRY(launch_check_digits(P, n, configs, status, st));
  if (t32 && n_sweeps > 0) HIP_TRY(launch_theta32(P, theta, t32, st));
  for (int k = 0; k < n_sweeps; ++k) {
    const uint64_t g = sweep0 + (uint64_t)k;
    if (k == 0) {
      s = compress_all_bots(P, n, theta, configs, w, status, trace, st);
      if (s != PEPS_OK) return s;
    }
    for (int r = 0; r < P.L1; ++r) {
      TIMED(PEPS_K_MOVES1, launch_moves1(P, n, r, theta, t32, configs, seed, g, sweep_counter, w, n_accept, status, st));
      if (r < P.L1 - 1) {
        TIMED(PEPS_K_MOVES2, launch_moves2(P, n, r, theta, t32, configs, seed, g, sweep_counter, w, n_accept, status, st));
        TIMED(PEPS_K_COMPRESS, compress_row(P, n, 0, r, theta, configs, w, status, st));
      }
    }
    if (k + 1 < n_sweeps || measure_any) {
      s = compress_all_bots(P, n, theta, configs, w, status, trace, st);
      if (s != PEPS_OK) return s;
    }
    if (measure_any) {
      const int64_t off = (int64_t)k * n;
      s = measure(P, n, theta, t32, configs, w, log_abs, sign, e_loc, O_rows ? O_rows + off * P.nnz : nullptr, off,
                  status, trace, st);
      if (s != PEPS_OK) return s;
      if (sample_configs)
        HIP_TRY(launch_copy_bytes(sample_configs + off * P.N, configs, (int64_t)n * P.N, st));
    }
  }
  if (sweep_counter && n_sweeps > 0) HIP_TRY(launch_advance_counter(sweep_counter, (uint64_t)n_sweeps, st));
  return PEPS_OK;
}

peps_status sr_cg_solve(const peps_desc* d, int64_t n_s, const uint8_t* configs, const double* O_rows,
                        const double* weights, const double* log_abs, const double* e_loc, double tau, double eps,
                        int32_t max_iter, double rtol, double* dtheta, double* g_out, double* theta, double* stats,
                        int32_t* status, void* ws, size_t ws_bytes, peps_trace* trace, peps_stream_t stream) {
  if (!desc_ok(d)) return PEPS_ERR_ARG;
  Prob P = make_prob(d);
  if (n_s < 1 || max_iter < 0 || max_iter > SR_MAX_ITER || !isfinite(tau) || !isfinite(eps) || eps < 0.0 ||
      !(rtol >= 0.0))
    return PEPS_ERR_ARG;
  if (!configs || !O_rows || !e_loc || !dtheta || !stats || !ws) return PEPS_ERR_ARG;
  size_t need = sr_workspace_bytes(P, n_s);
  if (ws_bytes < need) return PEPS_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_check_digits(P, n_s, configs, status, st));
  TIMED(PEPS_K_SR, launch_sr(P, n_s, configs, O_rows, weights, log_abs, e_loc, tau, eps, max_iter, rtol, dtheta,
                             g_out, theta, stats, status, ws, st));
  return PEPS_OK;
}

peps_status sr_cg_solve_noalloc(const peps_desc* d, int64_t n_s, const uint8_t* configs, const double* O_rows,
                                const double* weights, const double* log_abs, const double* e_loc, double tau,
                                double eps, int32_t max_iter, double rtol, double* dtheta, double* g_out,
                                double* theta, double* stats, int32_t* status, peps_stream_t stream) {
  if (!desc_ok(d)) return PEPS_ERR_ARG;
  Prob P = make_prob(d);
  if (n_s < 1 || max_iter < 0 || max_iter > SR_MAX_ITER || !isfinite(tau) || !isfinite(eps) || eps < 0.0 ||
      !(rtol >= 0.0))
    return PEPS_ERR_ARG;
  if (!configs || !O_rows || !e_loc || !dtheta || !stats) return PEPS_ERR_ARG;
  if (sr_workspace_bytes(P, n_s) > SR_STATIC_BYTES) return PEPS_ERR_WORKSPACE;
  void* ws = sr_static_scratch();
  if (!ws) return PEPS_ERR_HIP;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_check_digits(P, n_s, configs, status, st));
  HIP_TRY(launch_sr(P, n_s, configs, O_rows, weights, log_abs, e_loc, tau, eps, max_iter, rtol, dtheta, g_out, theta,
                    stats, status, ws, st));
  return PEPS_OK;
}

peps_status peps_sample_stats(const peps_desc* d, int32_t n_sweeps, int32_t n_chains, int32_t k,
                              const double* values, const double* weights, const double* log_abs, double* out,
                              peps_stream_t stream) {
  if (!desc_ok(d)) return PEPS_ERR_ARG;
  if (n_sweeps < 1 || n_chains < 1 || k < 1 || k > 4096) return PEPS_ERR_ARG;
  if (!values || !out) return PEPS_ERR_ARG;
  HIP_TRY(launch_sample_stats(make_prob(d), n_sweeps, n_chains, k, values, weights, log_abs, out,
                              (hipStream_t)stream));
  return PEPS_OK;
}

peps_status peps_vjp_batch(const peps_desc* d, int64_t n, const uint8_t* configs, const double* O_rows,
                           const double* cot, double* grad, void* ws, size_t ws_bytes, peps_stream_t stream) {
  if (!desc_ok(d)) return PEPS_ERR_ARG;
  Prob P = make_prob(d);
  if (n < 1) return PEPS_ERR_ARG;
  if (!configs || !O_rows || !cot || !grad || !ws) return PEPS_ERR_ARG;
  if (ws_bytes < sr_workspace_bytes(P, n)) return PEPS_ERR_WORKSPACE;
  HIP_TRY(launch_vjp(P, n, configs, O_rows, cot, grad, ws, (hipStream_t)stream));
  return PEPS_OK;
}

peps_status peps_observables_batch(const peps_desc* d, int64_t n, const uint8_t* configs, double* out,
                                   peps_stream_t stream) {
  if (!desc_ok(d)) return PEPS_ERR_ARG;
  if (n < 0) return PEPS_ERR_ARG;
  if (n == 0) return PEPS_OK;
  if (!configs || !out) return PEPS_ERR_ARG;
  Prob P = make_prob(d);
  HIP_TRY(launch_observables(P, n, configs, out, (hipStream_t)stream));
  return PEPS_OK;
}

static bool su_supported(const peps_desc* d) {
  return d->model == PEPS_MODEL_HEISENBERG && d->J2 == 0.0 && d->D <= MAX_SU_D;
}

peps_status peps_simple_update(const peps_desc* d, double* theta, double* lambdas, double tau, int32_t n_steps,
                               int32_t* status, void* ws, size_t ws_bytes, peps_stream_t stream) {
  if (!desc_ok(d) || n_steps < 0 || !isfinite(tau)) return PEPS_ERR_ARG;
  if (!su_supported(d)) return PEPS_ERR_UNSUPPORTED;
  if (n_steps == 0) return PEPS_OK;
  if (!theta || !lambdas || !ws) return PEPS_ERR_ARG;
  Prob P = make_prob(d);
  size_t need = 0;
  peps_workspace_bytes(d, 0, PEPS_WS_SU, &need);
  if (ws_bytes < need) return PEPS_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  for (int s = 0; s < n_steps; ++s) HIP_TRY(launch_su_step(P, theta, lambdas, tau, (double*)ws, status, st));
  return PEPS_OK;
}

peps_status peps_su_absorb(const peps_desc* d, const double* theta, const double* lambdas, double* theta_out,
                           peps_stream_t stream) {
  if (!desc_ok(d)) return PEPS_ERR_ARG;
  if (!su_supported(d)) return PEPS_ERR_UNSUPPORTED;
  if (!theta || !lambdas || !theta_out) return PEPS_ERR_ARG;
  Prob P = make_prob(d);
  HIP_TRY(launch_su_absorb(P, theta, lambdas, theta_out, (hipStream_t)stream));
  return PEPS_OK;
}

// ---- launch tuning ----------------------------------------------------------

peps_status peps_autotune_compression(const peps_desc* d, const double* theta, int32_t n, const uint8_t* configs,
                                      int32_t repeats, double* ms, int32_t* best, int32_t* status, void* ws,
                                      size_t ws_bytes, peps_stream_t stream) {
  if (!desc_ok(d) || n < 1 || n > (1 << 24) || repeats < 1 || repeats > 100) return PEPS_ERR_ARG;
  if (!theta || !configs || !ms || !best || !ws) return PEPS_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  Prob cand[4];
  bool ok[4] = {false, false, false, false};
  for (int k = PEPS_COMPRESS_REGISTER; k <= PEPS_COMPRESS_WORKSPACE; ++k) {
    peps_desc dk = *d;
    dk.compress_kernel = k;
    cand[k] = make_prob(&dk);
    ok[k] = device_support(&dk, cand[k]) == PEPS_OK;
    if (ok[k] && ws_bytes < chain_ws_bytes(cand[k], n)) return PEPS_ERR_WORKSPACE;
  }
  ms[0] = -1.0;
  *best = 0;
  double best_ms = 0.0;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return PEPS_ERR_HIP;
  }
  peps_status s = PEPS_OK;
  double* w = (double*)ws;
  for (int k = PEPS_COMPRESS_REGISTER; k <= PEPS_COMPRESS_WORKSPACE && s == PEPS_OK; ++k) {
    ms[k] = -1.0;
    if (!ok[k]) continue;
    const Prob& P = cand[k];
    auto pass = [&]() -> hipError_t {
      for (int r = 0; r <= P.L1 - 2; ++r) {
        hipError_t e = compress_row(P, n, 0, r, theta, configs, w, status, st);
        if (e != hipSuccess) return e;
      }
      for (int r = P.L1 - 1; r >= 1; --r) {
        hipError_t e = compress_row(P, n, 1, r, theta, configs, w, status, st);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    };
    float t = 0.f;
    if (launch_check_digits(P, n, configs, status, st) != hipSuccess || pass() != hipSuccess ||
        hipEventRecord(e0, st) != hipSuccess) {
      s = PEPS_ERR_HIP;
      break;
    }
    for (int i = 0; i < repeats && s == PEPS_OK; ++i)
      if (pass() != hipSuccess) s = PEPS_ERR_HIP;
    if (s != PEPS_OK || hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
      s = PEPS_ERR_HIP;
      break;
    }
    ms[k] = (double)t / repeats;
    if (*best == 0 || ms[k] < best_ms) {
      *best = k;
      best_ms = ms[k];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return s;
}

// ---- direct sampling (Appendix A) ------------------------------------------

// The chain problem (FP64 strips), the double layer's problem (one digit,
// bond D^2, boundary chi_dl) and the draw kernel's scratch layout.
static peps_status direct_setup(const peps_desc* d, int32_t chi_dl, Prob& P, Prob& Q, DirectLayout& L) {
  if (!desc_ok(d) || chi_dl < 1) return PEPS_ERR_ARG;
  peps_desc dp = *d;
  dp.precision = PEPS_PREC_FP64;
  P = make_prob(&dp);
  peps_status s = device_support(&dp, P);
  if (s != PEPS_OK) return s;
  peps_desc dq = dp;
  dq.d = 1;
  dq.D = d->D * d->D;
  dq.chi = chi_dl;
  dq.fermionic = 0;
  dq.compress_kernel = PEPS_COMPRESS_AUTO;
  Q = make_prob(&dq);
  s = device_support(&dq, Q);
  if (s != PEPS_OK) return s;
  L = direct_layout(P, Q);
  if ((int64_t)P.chi * P.chi > 255 * 255 || L.x1 > ((int64_t)1 << 24)) return PEPS_ERR_UNSUPPORTED;
  return PEPS_OK;
}

// Byte offsets of the regions of a direct-sampling workspace: the chains'
// boundary workspaces, the double-layer tensors, the double layer's
// one-chain workspace, its all-zero configuration, the draw scratch.
// The double layer (theta only) comes first, at offsets that do not depend
// on the number of chains, so that a later call may reuse it.
struct DirectRegions {
  size_t eth, wsq, cfgq, w, dws, total;
};
static DirectRegions direct_regions(const Prob& P, const Prob& Q, const DirectLayout& L, int64_t n) {
  auto pad = [](size_t x) { return (x + 255) & ~(size_t)255; };
  DirectRegions g;
  size_t off = 0;
  g.eth = off;  off += pad((size_t)Q.np * sizeof(double));
  g.wsq = off;  off += pad((size_t)Q.chain_stride * sizeof(double));
  g.cfgq = off; off += pad((size_t)P.N);
  g.w = off;    off += pad((size_t)n * P.chain_stride * sizeof(double));
  g.dws = off;  off += (size_t)n * L.stride * sizeof(double);
  g.total = off;
  return g;
}

peps_status peps_direct_workspace_bytes(const peps_desc* d, int64_t n_chains, int32_t chi_dl, size_t* bytes) {
  if (!bytes || n_chains < 0) return PEPS_ERR_ARG;
  Prob P, Q;
  DirectLayout L;
  peps_status s = direct_setup(d, chi_dl, P, Q, L);
  if (s != PEPS_OK) return s;
  *bytes = direct_regions(P, Q, L, n_chains).total;
  return PEPS_OK;
}

peps_status peps_direct_sample(const peps_desc* d, const double* theta, int32_t n_chains, int32_t chi_dl,
                               uint64_t seed, uint64_t draw, int32_t reweight, double* b_diag, int32_t update_b,
                               int32_t reuse_double_layer, uint8_t* configs, double* log_p, int32_t* status,
                               void* ws, size_t ws_bytes, peps_trace* trace, peps_stream_t stream) {
  if (n_chains < 0 || n_chains > (1 << 24)) return PEPS_ERR_ARG;
  if ((reweight != 0 && reweight != 1) || (update_b != 0 && update_b != 1)) return PEPS_ERR_ARG;
  if (reuse_double_layer != 0 && reuse_double_layer != 1) return PEPS_ERR_ARG;
  Prob P, Q;
  DirectLayout L;
  peps_status s = direct_setup(d, chi_dl, P, Q, L);
  if (s != PEPS_OK) return s;
  if (n_chains == 0) return PEPS_OK;
  if (!theta || !configs || !log_p || !ws || ((reweight || update_b) && !b_diag)) return PEPS_ERR_ARG;
  const DirectRegions g = direct_regions(P, Q, L, n_chains);
  if (ws_bytes < g.total) return PEPS_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  double* w = (double*)(base + g.w);
  double* eth = (double*)(base + g.eth);
  double* wsq = (double*)(base + g.wsq);
  uint8_t* cfgq = (uint8_t*)(base + g.cfgq);
  double* dws = (double*)(base + g.dws);
  const int n = n_chains;
  if (!reuse_double_layer) {
    TIMED(PEPS_K_DIRECT, launch_double_layer(P, Q, theta, eth, cfgq, st));
    for (int r = P.L1 - 1; r >= 1; --r) TIMED(PEPS_K_COMPRESS, compress_row(Q, 1, 1, r, eth, cfgq, wsq, status, st));
  }
  for (int r = 0; r < P.L1; ++r) {
    TIMED(PEPS_K_DIRECT, launch_direct_row(P, Q, L, n, r, theta, eth, configs, w, wsq, dws, seed, draw, reweight,
                                           b_diag, log_p, status, st));
    if (r < P.L1 - 1) TIMED(PEPS_K_COMPRESS, compress_row(P, n, 0, r, theta, configs, w, status, st));
  }
  if (update_b) TIMED(PEPS_K_DIRECT, launch_update_b(P, n, configs, b_diag, st));
  return PEPS_OK;
}

peps_status peps_importance_weights(int64_t n, const double* log_abs, const double* log_p, double* weights,
                                    peps_stream_t stream) {
  if (n < 1 || n > ((int64_t)1 << 30) || !log_abs || !log_p || !weights) return PEPS_ERR_ARG;
  HIP_TRY(launch_importance_weights(n, log_abs, log_p, weights, (hipStream_t)stream));
  return PEPS_OK;
}

peps_trace* peps_trace_create(int32_t capacity) {
  if (capacity < 1) return nullptr;
  peps_trace* t = new peps_trace;
  t->capacity = capacity;
  t->a.assign(capacity, nullptr);
  t->b.assign(capacity, nullptr);
  t->cls.assign(capacity, 0);
  t->notes.assign(capacity, peps_trace::Note{nullptr, nullptr, 0, 0});
  for (int i = 0; i < capacity; ++i) {
    if (hipEventCreate(&t->a[i]) != hipSuccess || hipEventCreate(&t->b[i]) != hipSuccess) {
      peps_trace_destroy(t);
      return nullptr;
    }
  }
  return t;
}

void peps_trace_destroy(peps_trace* t) {
  if (!t) return;
  for (auto e : t->a)
    if (e) (void)hipEventDestroy(e);
  for (auto e : t->b)
    if (e) (void)hipEventDestroy(e);
  delete t;
}

void peps_progress_stderr(void* user, int32_t kernel_class, int32_t launch) {
  // seconds since the first line this process printed
  static const auto t0 = std::chrono::steady_clock::now();
  const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  fprintf(stderr, "[peps] %s class %d launch %d done (%.1f s)\n", user ? (const char*)user : "", (int)kernel_class,
          (int)launch, t);
  fflush(stderr);
}

peps_status peps_trace_set_progress(peps_trace* t, peps_progress_fn fn, void* user) {
  if (!t) return PEPS_ERR_ARG;
  t->fn = fn;
  t->user = user;
  return PEPS_OK;
}

peps_status peps_trace_read(peps_trace* t, double* ms, int64_t* launches) {
  if (!t) return PEPS_ERR_ARG;
  peps_status s = PEPS_OK;
  for (int i = 0; i < t->used; ++i) {
    float v = 0.f;
    if (hipEventSynchronize(t->b[i]) != hipSuccess || hipEventElapsedTime(&v, t->a[i], t->b[i]) != hipSuccess) {
      s = PEPS_ERR_HIP;
      continue;
    }
    const int c = t->cls[i];
    if (ms) ms[c] += v;
    if (launches) launches[c] += 1;
  }
  t->used = 0;
  return s;
}

}  // extern "C"
