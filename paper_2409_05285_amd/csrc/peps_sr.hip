// Stochastic reconfiguration on the GPU (FP64): sample reductions and the
// conjugate-gradient solve of (S + eps 1) dtheta = -tau g with the metric
// applied as O^T (O x - mean(O x)), never formed.
//
// O is stored compressed, one block per site and sample; the parameter
// index of entry e of sample i is  base[e] + S_i[site[e]] * bsz[e].
//   gather  y_i = O_i . x  : GR sample rows per workgroup, coalesced along e;
//   scatter z = O^T t      : one thread per column e and chunk of samples,
//                            d^2 register accumulators selected by S_i, then a
//                            fixed-order sum over chunks.
// Every reduction has a fixed shape, so results are bit-identical run to run.
#include <math.h>

#include <mutex>

#include "peps_common.hpp"
#include "peps_kernels.hpp"

namespace peps {

// Scratch of the solve that allocates nothing (sr_cg_solve_noalloc): one
// fixed device array per GPU, reserved when the code object is loaded.  In
// host code `scratch` names a host-side stand-in, never the device memory:
// the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) char scratch[SR_STATIC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

void* sr_static_scratch() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

constexpr int SR_NT = 256;
constexpr int YB = 128;   // blocks of the weighted mean of y

struct SrDev {
  int64_t n_s, nnz, np;
  int N, d2, n_chunks, rows_per_chunk, n_red;  // n_red: blocks of the vector kernels
  const uint8_t* configs;
  const double* O;
  const double* e;
  const int32_t* base;   // [nnz]
  const int32_t* bsz;    // [nnz]
  const int32_t* site;   // [nnz]
  const int32_t* soff;   // [N] O-row offset of each site
  const int32_t* spoff;  // [N] parameter offset of each site
  const int32_t* sbs;    // [N] block size of each site
  double* w;             // [n_s] normalised weights
  double* y;             // [n_s]
  double* zpart;         // [n_chunks][np]
  double* r;
  double* p;
  double* Ap;
  double* x;
  double* g;
  double* part;          // [2][n_red]
  double* ypart;         // [YB] block partials of sum_i w_i y_i
  double* scal;          // [max_iter + 2][4]: rr, stop, pAp, alpha
  double* misc;          // [8]: ebar, bnorm, ybar, ...
};

__device__ inline double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = SR_NT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  double out = red[0];
  __syncthreads();
  return out;
}

// Weights and Ebar (single block).  Explicit weights when given; else
// |rho_i|^(2 - alpha) from the log-amplitudes (relative to the largest)
// when given and alpha != 2; else uniform.
__global__ void __launch_bounds__(SR_NT) k_sr_weights(SrDev D, const double* weights, const double* log_abs,
                                                       int alpha) {
  __shared__ double red[SR_NT];
  const int tid = threadIdx.x;
  const bool from_la = weights == nullptr && log_abs != nullptr && alpha != 2;
  double lmax = -INFINITY;
  if (from_la) {
    for (int64_t i = tid; i < D.n_s; i += SR_NT) lmax = fmax(lmax, log_abs[i]);
    red[tid] = lmax;
    __syncthreads();
    for (int s = SR_NT / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
      __syncthreads();
    }
    lmax = red[0];
    __syncthreads();
  }
  auto raw = [&](int64_t i) {
    return weights ? weights[i] : exp((double)(2 - alpha) * (log_abs[i] - lmax));
  };
  const bool nonuniform = weights != nullptr || from_la;
  double ws = 0.0;
  if (nonuniform) {
    for (int64_t i = tid; i < D.n_s; i += SR_NT) ws += raw(i);
    ws = block_sum(ws, red);
  }
  double es = 0.0;
  for (int64_t i = tid; i < D.n_s; i += SR_NT) {
    double wi = nonuniform ? raw(i) / ws : 1.0 / (double)D.n_s;
    D.w[i] = wi;
    es += wi * D.e[i];
  }
  es = block_sum(es, red);
  if (tid == 0) {
    D.misc[0] = es;
    D.misc[4] = 0.0;  // breakdown flag
  }
}

// Weighted mean of y in two fixed-order stages: block b sums its slice of
// w_i y_i into ypart[b]; the scatter kernel adds the YB partials.
__global__ void __launch_bounds__(SR_NT) k_sr_ymean(SrDev D, int it) {
  __shared__ double red[SR_NT];
  if (it >= 0 && D.scal[it * 4 + 1] != 0.0) return;
  const int64_t per = (D.n_s + YB - 1) / YB;
  const int64_t i0 = (int64_t)blockIdx.x * per;
  const int64_t i1 = i0 + per < D.n_s ? i0 + per : D.n_s;
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += SR_NT) s += D.w[i] * D.y[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) D.ypart[blockIdx.x] = s;
}

// y_i = O_i . v for GR sample rows per workgroup.  Threads stride over the
// entries e of a row (coalesced reads of O).  Entry e of site s maps to the
// parameter spoff[s] + S_i[s] sbs[s] + (e - soff[s]); the per-row offsets are
// staged in LDS and each thread follows its site with a running index (its
// entries increase).  Per-thread partial sums, then a fixed-order wave and
// workgroup reduction.
constexpr int GR = 2;
__global__ void __launch_bounds__(SR_NT) k_sr_gather(SrDev D, const double* v, int it) {
  __shared__ int soff[MAX_SITES + 1];
  __shared__ int vb[GR][MAX_SITES];
  __shared__ double red[SR_NT / 64][GR];
  if (it >= 0 && D.scal[it * 4 + 1] != 0.0) return;
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * GR;
  const int nr = D.n_s - row0 < GR ? (int)(D.n_s - row0) : GR;
  for (int q = tid; q < GR * D.N; q += SR_NT) {
    const int r = q / D.N, st = q % D.N;
    const int Sv = r < nr ? D.configs[(row0 + r) * D.N + st] : 0;
    const int S = Sv < D.d2 ? Sv : 0;   // range-checked digit (see k_check_digits)
    vb[r][st] = D.spoff[st] + S * D.sbs[st] - D.soff[st];
  }
  for (int st = tid; st < D.N; st += SR_NT) soff[st] = D.soff[st];
  if (tid == 0) soff[D.N] = (int)D.nnz;
  __syncthreads();
  double acc[GR];
#pragma unroll
  for (int r = 0; r < GR; ++r) acc[r] = 0.0;
  int st = 0;
  int e = tid;
  // four entries per thread and pass, loads issued before the products
  // (same summation order as one entry per pass)
  constexpr int EU = 4;
  for (; e + (EU - 1) * SR_NT < D.nnz; e += EU * SR_NT) {
    int sts[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      while (e + u * SR_NT >= soff[st + 1]) ++st;
      sts[u] = st;
    }
    double o[EU][GR], x[EU][GR];
#pragma unroll
    for (int u = 0; u < EU; ++u)
#pragma unroll
      for (int r = 0; r < GR; ++r) {
        const int eu = e + u * SR_NT;
        o[u][r] = r < nr ? D.O[(row0 + r) * D.nnz + eu] : 0.0;
        x[u][r] = r < nr ? v[vb[r][sts[u]] + eu] : 0.0;
      }
#pragma unroll
    for (int u = 0; u < EU; ++u)
#pragma unroll
      for (int r = 0; r < GR; ++r)
        if (r < nr) acc[r] += o[u][r] * x[u][r];
  }
  for (; e < D.nnz; e += SR_NT) {
    while (e >= soff[st + 1]) ++st;
#pragma unroll
    for (int r = 0; r < GR; ++r)
      if (r < nr) acc[r] += D.O[(row0 + r) * D.nnz + e] * v[vb[r][st] + e];
  }
#pragma unroll
  for (int r = 0; r < GR; ++r)
    for (int off = 32; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off, 64);
  if ((tid & 63) == 0)
#pragma unroll
    for (int r = 0; r < GR; ++r) red[tid >> 6][r] = acc[r];
  __syncthreads();
  if (tid < nr) {
    double t = 0.0;
    for (int wv = 0; wv < SR_NT / 64; ++wv) t += red[wv][tid];
    D.y[row0 + tid] = t;
  }
}

// zpart[chunk][k] = sum_{i in chunk} t_i O_i[e] at k = base[e] + S_i * bsz[e],
// with t_i = w_i (src_i - mean): src = e_loc (mode 0, mean misc[0]) or
// y (mode 1, mean from the YB partials of k_sr_ymean); mode 2: t_i = e_i (the
// cotangent, no weights).
template <int D2>
__global__ void __launch_bounds__(SR_NT) k_sr_scatter(SrDev D, int mode, int it) {
  __shared__ double red[SR_NT];
  if (it >= 0 && D.scal[it * 4 + 1] != 0.0) return;
  double mean = mode == 0 ? D.misc[0] : 0.0;
  if (mode == 1) mean = block_sum(threadIdx.x < YB ? D.ypart[threadIdx.x] : 0.0, red);
  const int64_t e = (int64_t)blockIdx.x * SR_NT + threadIdx.x;
  const int chunk = blockIdx.y;
  if (e >= D.nnz) return;
  const double* src = mode == 1 ? D.y : D.e;
  const int st = D.site[e];
  double acc[D2];
#pragma unroll
  for (int q = 0; q < D2; ++q) acc[q] = 0.0;
  const int64_t i0 = (int64_t)chunk * D.rows_per_chunk;
  int64_t i1 = i0 + D.rows_per_chunk;
  if (i1 > D.n_s) i1 = D.n_s;
  int64_t i = i0;
  // eight rows per pass, loads issued before the accumulation (same order
  // of summation as one row per pass)
  constexpr int UR = 8;
  for (; i + UR <= i1; i += UR) {
    double o[UR], t[UR];
    int sv[UR];
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      o[u] = D.O[(i + u) * D.nnz + e];
      sv[u] = D.configs[(i + u) * D.N + st];
      t[u] = mode == 2 ? src[i + u] : D.w[i + u] * (src[i + u] - mean);
    }
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const double v = t[u] * o[u];
#pragma unroll
      for (int q = 0; q < D2; ++q) acc[q] += (sv[u] == q) ? v : 0.0;
    }
  }
  for (; i < i1; ++i) {
    const double t = mode == 2 ? src[i] : D.w[i] * (src[i] - mean);
    const double v = t * D.O[i * D.nnz + e];
    const int Si = D.configs[i * D.N + st];
#pragma unroll
    for (int q = 0; q < D2; ++q) acc[q] += (Si == q) ? v : 0.0;
  }
  double* zp = D.zpart + (int64_t)chunk * D.np;
  const int64_t b = D.base[e];
  const int bs = D.bsz[e];
#pragma unroll
  for (int q = 0; q < D2; ++q) zp[b + (int64_t)q * bs] = acc[q];
}

// Sum of the chunk partials.  mode 0: g = z, then CG start vectors
// b = -tau g: x = 0, r = p = b, part = partial(b.b).
// mode 1: Ap = z + eps p, part = partial(p.Ap).
// mode 2: g = z only (vector-Jacobian product).
__global__ void __launch_bounds__(SR_NT) k_sr_reduce(SrDev D, int mode, double tau, double eps, int it) {
  __shared__ double red[SR_NT];
  if (it >= 0 && D.scal[it * 4 + 1] != 0.0) return;
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * SR_NT + threadIdx.x; k < D.np; k += (int64_t)D.n_red * SR_NT) {
    double z = 0.0;
    for (int c = 0; c < D.n_chunks; ++c) z += D.zpart[(int64_t)c * D.np + k];
    if (mode == 2) {
      D.g[k] = z;
    } else if (mode == 0) {
      D.g[k] = z;
      const double b = -tau * z;
      D.x[k] = 0.0;
      D.r[k] = b;
      D.p[k] = b;
      s += b * b;
    } else {
      const double ap = z + eps * D.p[k];
      D.Ap[k] = ap;
      s += D.p[k] * ap;
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) D.part[blockIdx.x] = s;
}

__device__ inline double sum_parts(const double* part, int n, double* red) {
  double s = 0.0;
  for (int q = threadIdx.x; q < n; q += SR_NT) s += part[q];
  return block_sum(s, red);
}

// rr_0, ||b|| and the first stop flag (single block).
__global__ void __launch_bounds__(SR_NT) k_sr_start(SrDev D, double rtol, int max_iter) {
  __shared__ double red[SR_NT];
  const double rr = sum_parts(D.part, D.n_red, red);
  if (threadIdx.x == 0) {
    D.misc[1] = sqrt(rr);
    D.scal[0] = rr;
    D.scal[1] = (max_iter <= 0 || sqrt(rr) <= rtol * sqrt(rr)) ? 1.0 : 0.0;
  }
}

// x += alpha p, r -= alpha Ap, part2 = partial(r.r).  alpha = rr / pAp.
__global__ void __launch_bounds__(SR_NT) k_sr_update(SrDev D, int it, int32_t* status) {
  __shared__ double red[SR_NT];
  if (D.scal[it * 4 + 1] != 0.0) return;
  const double pAp = sum_parts(D.part, D.n_red, red);
  const double rr = D.scal[it * 4 + 0];
  if (!(pAp > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      D.scal[it * 4 + 2] = pAp;
      D.misc[4] = 1.0;
      set_status(status, PEPS_ERR_CG_BREAKDOWN);
    }
    return;
  }
  const double alpha = rr / pAp;
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * SR_NT + threadIdx.x; k < D.np; k += (int64_t)D.n_red * SR_NT) {
    D.x[k] += alpha * D.p[k];
    const double rk = D.r[k] - alpha * D.Ap[k];
    D.r[k] = rk;
    s += rk * rk;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) D.part[D.n_red + blockIdx.x] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    D.scal[it * 4 + 2] = pAp;
    D.scal[it * 4 + 3] = alpha;
  }
}

// p = r + beta p; scalars of iteration it+1.
__global__ void __launch_bounds__(SR_NT) k_sr_direction(SrDev D, int it, double rtol, int max_iter) {
  __shared__ double red[SR_NT];
  const bool stopped = D.scal[it * 4 + 1] != 0.0;
  if (stopped) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      D.scal[(it + 1) * 4 + 0] = D.scal[it * 4 + 0];
      D.scal[(it + 1) * 4 + 1] = D.scal[it * 4 + 1];
    }
    return;
  }
  if (!(D.scal[it * 4 + 2] > 0.0)) {  // breakdown: stop with the current x
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      D.scal[(it + 1) * 4 + 0] = D.scal[it * 4 + 0];
      D.scal[(it + 1) * 4 + 1] = 2.0;
    }
    return;
  }
  const double rr_new = sum_parts(D.part + D.n_red, D.n_red, red);
  const double beta = rr_new / D.scal[it * 4 + 0];
  for (int64_t k = (int64_t)blockIdx.x * SR_NT + threadIdx.x; k < D.np; k += (int64_t)D.n_red * SR_NT)
    D.p[k] = D.r[k] + beta * D.p[k];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    D.scal[(it + 1) * 4 + 0] = rr_new;
    D.scal[(it + 1) * 4 + 1] = (it + 1 >= max_iter || sqrt(rr_new) <= rtol * D.misc[1]) ? 1.0 : 0.0;
  }
}

// stats: Ebar, ||r||, iterations, ||b||, and 1 when max_iter iterations
// ended above the residual bar (also a warning in the status word).
__global__ void k_sr_stats(SrDev D, int max_iter, double rtol, double* stats, int32_t* status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int it = 0;
  while (it < max_iter && D.scal[it * 4 + 1] == 0.0) ++it;
  const double rn = sqrt(D.scal[it * 4 + 0]);
  const bool broke = D.misc[4] != 0.0;
  const bool not_conv = max_iter > 0 && !broke && it >= max_iter && !(rn <= rtol * D.misc[1]);
  stats[0] = D.misc[0];
  stats[1] = rn;
  stats[2] = (double)it;
  stats[3] = D.misc[1];
  stats[4] = not_conv ? 1.0 : 0.0;
  if (!isfinite(D.misc[0]) || !isfinite(D.misc[1])) set_status(status, PEPS_ERR_NONFINITE);
  if (not_conv) set_status(status, PEPS_WARN_CG_NOT_CONVERGED);
}

// theta += dtheta unless the solve broke down.
__global__ void __launch_bounds__(SR_NT) k_sr_apply(SrDev D, double* theta) {
  if (D.misc[4] != 0.0) return;
  for (int64_t k = (int64_t)blockIdx.x * SR_NT + threadIdx.x; k < D.np; k += (int64_t)D.n_red * SR_NT)
    theta[k] += D.x[k];
}

// Column maps of the compressed O rows.
__global__ void k_sr_colmap(Prob P, int32_t* base, int32_t* bsz, int32_t* site, int32_t* soff, int32_t* spoff,
                            int32_t* sbs) {
  __shared__ Geo geo;
  if (threadIdx.x == 0) build_geo(P, geo);
  __syncthreads();
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < P.N; i += blockDim.x) {
      soff[i] = geo.ooff[i];
      spoff[i] = geo.poff[i];
      sbs[i] = block_size(P, i / P.L2, i % P.L2);
    }
  for (int i = blockIdx.x; i < P.N; i += gridDim.x) {
    const int r = i / P.L2, c = i % P.L2;
    const int bs = block_size(P, r, c);
    for (int j = threadIdx.x; j < bs; j += blockDim.x) {
      const int e = geo.ooff[i] + j;
      base[e] = geo.poff[i] + j;
      bsz[e] = bs;
      site[e] = i;
    }
  }
}

// ---------------------------------------------------------------------------

static void sr_layout(const Prob& P, int64_t n_s, SrDev& D, size_t* bytes, char* ws) {
  D.n_s = n_s;
  D.nnz = P.nnz;
  D.np = P.np;
  D.N = P.N;
  D.d2 = P.d2;
  const int64_t cols_blocks = (P.nnz + SR_NT - 1) / SR_NT;
  int64_t chunks = (2048 + cols_blocks - 1) / cols_blocks;
  if (chunks > 64) chunks = 64;
  if (chunks < 1) chunks = 1;
  if (chunks > n_s) chunks = n_s > 0 ? n_s : 1;
  D.rows_per_chunk = (int)((n_s + chunks - 1) / chunks);
  D.n_chunks = (int)((n_s + D.rows_per_chunk - 1) / D.rows_per_chunk);
  if (D.n_chunks < 1) D.n_chunks = 1;
  int64_t nred = (P.np + SR_NT - 1) / SR_NT;
  D.n_red = (int)(nred > 1024 ? 1024 : (nred < 1 ? 1 : nred));
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += (b + 255) & ~(size_t)255; return o; };
  size_t o_base = take(sizeof(int32_t) * P.nnz), o_bsz = take(sizeof(int32_t) * P.nnz),
         o_site = take(sizeof(int32_t) * P.nnz);
  size_t o_soff = take(sizeof(int32_t) * P.N), o_spoff = take(sizeof(int32_t) * P.N),
         o_sbs = take(sizeof(int32_t) * P.N);
  size_t o_w = take(sizeof(double) * n_s), o_y = take(sizeof(double) * n_s);
  size_t o_z = take(sizeof(double) * (size_t)D.n_chunks * P.np);
  size_t o_r = take(sizeof(double) * P.np), o_p = take(sizeof(double) * P.np), o_ap = take(sizeof(double) * P.np);
  size_t o_g = take(sizeof(double) * P.np);
  size_t o_part = take(sizeof(double) * 2 * D.n_red);
  size_t o_scal = take(sizeof(double) * 4 * (size_t)(SR_MAX_ITER + 2));
  size_t o_misc = take(sizeof(double) * 8);
  size_t o_ypart = take(sizeof(double) * YB);
  *bytes = off;
  if (ws) {
    D.base = (const int32_t*)(ws + o_base);
    D.bsz = (const int32_t*)(ws + o_bsz);
    D.site = (const int32_t*)(ws + o_site);
    D.soff = (const int32_t*)(ws + o_soff);
    D.spoff = (const int32_t*)(ws + o_spoff);
    D.sbs = (const int32_t*)(ws + o_sbs);
    D.w = (double*)(ws + o_w);
    D.y = (double*)(ws + o_y);
    D.zpart = (double*)(ws + o_z);
    D.r = (double*)(ws + o_r);
    D.p = (double*)(ws + o_p);
    D.Ap = (double*)(ws + o_ap);
    D.g = (double*)(ws + o_g);
    D.part = (double*)(ws + o_part);
    D.scal = (double*)(ws + o_scal);
    D.misc = (double*)(ws + o_misc);
    D.ypart = (double*)(ws + o_ypart);
  }
}

size_t sr_workspace_bytes(const Prob& P, int64_t n_s) {
  SrDev D;
  size_t b = 0;
  sr_layout(P, n_s, D, &b, nullptr);
  return b;
}

hipError_t launch_sr(const Prob& P, int64_t n_s, const uint8_t* configs, const double* O, const double* weights,
                     const double* log_abs, const double* e_loc, double tau, double eps, int max_iter, double rtol, double* dtheta,
                     double* g_out, double* theta, double* stats, int32_t* status, void* ws, hipStream_t st) {
  SrDev D;
  size_t b = 0;
  sr_layout(P, n_s, D, &b, (char*)ws);
  D.configs = configs;
  D.O = O;
  D.e = e_loc;
  D.x = dtheta;
  if (g_out) D.g = g_out;
  const int cb = (int)((P.nnz + SR_NT - 1) / SR_NT);
  hipLaunchKernelGGL(k_sr_colmap, dim3(P.N < 1024 ? P.N : 1024), dim3(256), 0, st, P, (int32_t*)D.base,
                     (int32_t*)D.bsz, (int32_t*)D.site, (int32_t*)D.soff, (int32_t*)D.spoff, (int32_t*)D.sbs);
  hipLaunchKernelGGL(k_sr_weights, dim3(1), dim3(SR_NT), 0, st, D, weights, log_abs, P.alpha);
  auto scatter = [&](int mode, int it) {
    if (P.d2 == 4)
      hipLaunchKernelGGL(k_sr_scatter<4>, dim3(cb, D.n_chunks), dim3(SR_NT), 0, st, D, mode, it);
    else
      hipLaunchKernelGGL(k_sr_scatter<16>, dim3(cb, D.n_chunks), dim3(SR_NT), 0, st, D, mode, it);
  };
  scatter(0, -1);
  hipLaunchKernelGGL(k_sr_reduce, dim3(D.n_red), dim3(SR_NT), 0, st, D, 0, tau, eps, -1);
  hipLaunchKernelGGL(k_sr_start, dim3(1), dim3(SR_NT), 0, st, D, rtol, max_iter);
  const int gb = (int)((n_s + GR - 1) / GR);
  for (int it = 0; it < max_iter; ++it) {
    hipLaunchKernelGGL(k_sr_gather, dim3(gb), dim3(SR_NT), 0, st, D, (const double*)D.p, it);
    hipLaunchKernelGGL(k_sr_ymean, dim3(YB), dim3(SR_NT), 0, st, D, it);
    scatter(1, it);
    hipLaunchKernelGGL(k_sr_reduce, dim3(D.n_red), dim3(SR_NT), 0, st, D, 1, tau, eps, it);
    hipLaunchKernelGGL(k_sr_update, dim3(D.n_red), dim3(SR_NT), 0, st, D, it, status);
    hipLaunchKernelGGL(k_sr_direction, dim3(D.n_red), dim3(SR_NT), 0, st, D, it, rtol, max_iter);
  }
  hipLaunchKernelGGL(k_sr_stats, dim3(1), dim3(64), 0, st, D, max_iter, rtol, stats, status);
  if (theta) hipLaunchKernelGGL(k_sr_apply, dim3(D.n_red), dim3(SR_NT), 0, st, D, theta);
  return hipGetLastError();
}

// grad = sum_i cot_i O_i, scattered into the parameter layout.
hipError_t launch_vjp(const Prob& P, int64_t n_s, const uint8_t* configs, const double* O, const double* cot,
                      double* grad, void* ws, hipStream_t st) {
  SrDev D;
  size_t b = 0;
  sr_layout(P, n_s, D, &b, (char*)ws);
  D.configs = configs;
  D.O = O;
  D.e = cot;
  D.g = grad;
  const int cb = (int)((P.nnz + SR_NT - 1) / SR_NT);
  hipLaunchKernelGGL(k_sr_colmap, dim3(P.N < 1024 ? P.N : 1024), dim3(256), 0, st, P, (int32_t*)D.base,
                     (int32_t*)D.bsz, (int32_t*)D.site, (int32_t*)D.soff, (int32_t*)D.spoff, (int32_t*)D.sbs);
  if (P.d2 == 4)
    hipLaunchKernelGGL(k_sr_scatter<4>, dim3(cb, D.n_chunks), dim3(SR_NT), 0, st, D, 2, -1);
  else
    hipLaunchKernelGGL(k_sr_scatter<16>, dim3(cb, D.n_chunks), dim3(SR_NT), 0, st, D, 2, -1);
  hipLaunchKernelGGL(k_sr_reduce, dim3(D.n_red), dim3(SR_NT), 0, st, D, 2, 0.0, 0.0, -1);
  return hipGetLastError();
}

}  // namespace peps
