// Boundary-row compression, register-resident version (one workgroup of 512
// threads per chain).
//
//   1. absorb the row into the boundary: B_c[(a,l)][p][(b,r)];
//   2. left-to-right thin Householder QR with the matrix in registers (wave w
//      owns 8 columns, lane l four rows), one workgroup barrier per
//      reflector; R is kept in LDS and R B_{c+1} is formed straight into the
//      registers of the next step (rows (x, p) of the next matrix, p fastest);
//   3. right-to-left truncation by one-sided Jacobi in LDS: G = M^T when M is
//      wide or square (no accumulation; U S = M V_k afterwards), G = M with an
//      accumulated V when M is tall;
//   4. normalisation and log-scale.
// Supported shapes: matrices up to 256 x 64 in the QR sweep, 64 x 64 in the
// truncation (chi * D <= 64), physical dimension D in {1, 2, 4}.
#include <math.h>

#include "peps_common.hpp"
#include "peps_kernels.hpp"

namespace peps {

namespace {

constexpr int NTC = 512;        // threads per workgroup (8 waves)
constexpr int QR_RPL = 4;       // rows per lane (64 lanes x 4 = 256 rows)
constexpr int QR_CPW = 8;       // columns per wave (8 waves x 8 = 64 columns)
constexpr int QR_ROWS_MAX = 256;
static_assert(QR_RPL % 4 == 0, "rows per lane must be a multiple of every supported D");
constexpr int QR_COLS = 64;     // max columns
constexpr int SV_MAX = 64;      // max truncation matrix dimension
constexpr int SV_LD = SV_MAX + 1;
constexpr int JL = 16;          // lanes per Jacobi pair
constexpr int JR = SV_MAX / JL; // rows per lane
constexpr int JAC_MAX_SWEEPS_V2 = 40;
constexpr double JAC_TOL = 2.0e-15;

struct ChainPtrs {
  double *top, *lstop, *bot, *lsbot, *B;
};

__device__ inline ChainPtrs chain_ptrs(const Prob& P, double* ws, int ch) {
  double* base = ws + (size_t)ch * P.chain_stride;
  ChainPtrs w;
  w.top = base + P.off_top;
  w.lstop = base + P.off_lstop;
  w.bot = base + P.off_bot;
  w.lsbot = base + P.off_lsbot;
  w.B = base + P.off_B;
  return w;
}

// fixed-order sum of NTC values through LDS, identical on every thread
__device__ inline double block_sum512(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = NTC / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// 1/x and 1/sqrt(x) from the hardware estimates refined by Newton steps
// (each step doubles the correct bits; two reach double precision), and
// sqrt(1 + x^2) as y * rsqrt(y).  Used for the Jacobi rotation parameters,
// where a few ulp only perturb orthogonality at rounding level.
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ inline double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r;
}
__device__ inline double sqrt1p_sq(double a) {
  const double y = fma(a, a, 1.0);
  return y * rsqrt_nr(y);
}

// Lane exchange inside one 16-lane DPP row, for a double.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a DPP row.  Each stage adds a value and its
// mirror partner (xor 1, xor 2 in quads, then half-row and row mirrors), so
// every lane ends with the same bits.
__device__ inline double row16_sum(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);   // row_half_mirror
  v += dpp_f64<0x140>(v);   // row_mirror
  return v;
}


// Sum over the 64 lanes of a wave with identical bits on every lane:
// mirror-pair stages inside each 16-lane row, then xor 16 and xor 32.
__device__ inline double wave_sum(double v) {
  v = row16_sum(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// One-sided Jacobi on G (mg x ng <= 64 x 64, column-major, stride SV_LD),
// optionally accumulating V (ng x ng, column-major, stride SV_LD).
__device__ void jacobi64(double* G, int mg, int ng, double* V, int* flags) {
  const int tid = threadIdx.x;
  if (ng < 2) return;
  const int ne = ng + (ng & 1);
  const int npairs = ne / 2;
  const int grp = tid / JL, lane = tid % JL;
  if (tid == 0) { flags[0] = 0; flags[1] = 0; }
  __syncthreads();
  for (int sweep = 0; sweep < JAC_MAX_SWEEPS_V2; ++sweep) {
    const int fl = sweep & 1;
    for (int rnd = 0; rnd < ne - 1; ++rnd) {
      int ci = -1, cj = -1;
      if (grp < npairs) {
        if (grp == 0) { ci = rnd; cj = ne - 1; }
        else { ci = (rnd + grp) % (ne - 1); cj = (rnd - grp + ne - 1) % (ne - 1); }
        if (ci >= ng || cj >= ng) ci = -1;
        if (ci > cj && ci >= 0) { int t = ci; ci = cj; cj = t; }
      }
      double x[JR], y[JR];
      double al = 0.0, be = 0.0, ga = 0.0;
      if (ci >= 0) {
        const double* gi = G + ci * SV_LD;
        const double* gj = G + cj * SV_LD;
#pragma unroll
        for (int t = 0; t < JR; ++t) {
          const int i = lane + JL * t;
          x[t] = i < mg ? gi[i] : 0.0;
          y[t] = i < mg ? gj[i] : 0.0;
          al += x[t] * x[t];
          be += y[t] * y[t];
          ga += x[t] * y[t];
        }
      }
      al = row16_sum(al);
      be = row16_sum(be);
      ga = row16_sum(ga);
      if (ci >= 0 && ga != 0.0 && ga * ga > (JAC_TOL * JAC_TOL) * (al * be)) {
        const double zeta = (be - al) * rcp_nr(2.0 * ga);
        const double az = fabs(zeta);
        const double root = az < 1.0e150 ? sqrt1p_sq(az) : az;
        const double t = copysign(rcp_nr(az + root), zeta);
        const double c = rsqrt_nr(fma(t, t, 1.0));
        const double s = c * t;
        double* gi = G + ci * SV_LD;
        double* gj = G + cj * SV_LD;
#pragma unroll
        for (int tt = 0; tt < JR; ++tt) {
          const int i = lane + JL * tt;
          if (i < mg) {
            gi[i] = c * x[tt] - s * y[tt];
            gj[i] = s * x[tt] + c * y[tt];
          }
        }
        if (V) {
          double* vi = V + ci * SV_LD;
          double* vj = V + cj * SV_LD;
#pragma unroll
          for (int tt = 0; tt < JR; ++tt) {
            const int i = lane + JL * tt;
            if (i < ng) {
              const double a = vi[i], b = vj[i];
              vi[i] = c * a - s * b;
              vj[i] = s * a + c * b;
            }
          }
        }
        if (lane == 0) flags[fl] = 1;
      }
      __syncthreads();
    }
    const bool done = flags[fl] == 0;
    __syncthreads();
    if (tid == 0) flags[fl] = 0;
    __syncthreads();
    if (done) break;
  }
}

}  // namespace

template <int DP>
__global__ void __launch_bounds__(NTC, 4) k_compress2(Prob P, int dir, int r, const double* __restrict__ theta,
                                                     const uint8_t* __restrict__ configs, double* ws,
                                                     int32_t* status) {
  __shared__ double qv[2][QR_ROWS_MAX];
  __shared__ double qtau[2];
  __shared__ double taus[QR_COLS];
  __shared__ double red[NTC];
  __shared__ double bufA[QR_COLS * SV_LD];   // R during the QR sweep; G during truncation
  __shared__ double bufB[QR_COLS * SV_LD];   // V / U S during truncation
  __shared__ int sa[MAX_L], sp[MAX_L], sb[MAX_L];
  __shared__ int pa[MAX_L], pb[MAX_L], oa[MAX_L], ob[MAX_L], poffr[MAX_L];
  __shared__ int flags[2];
  __shared__ int bad;
  __shared__ double alpha_sh[2];
  __shared__ int ta[MAX_L], tb[MAX_L], tp[MAX_L];
  __shared__ double sig[SV_MAX];
  __shared__ int rnk[SV_MAX];

  const int tid = threadIdx.x;
  const int ch = blockIdx.x;
  ChainPtrs w = chain_ptrs(P, ws, ch);
  const uint8_t* cfg = configs + (size_t)ch * P.N;
  double* bnd = dir == 0 ? w.top : w.bot;
  double* lsb = dir == 0 ? w.lstop : w.lsbot;
  double* outT = bnd + (size_t)r * P.L2 * P.TS;
  const bool has_prev = dir == 0 ? (r > 0) : (r < P.L1 - 1);
  const int rp = dir == 0 ? r - 1 : r + 1;

  if (tid == 0) {
    // static dims of the previous boundary row and of the output row
    int* a = ta;
    int* b = tb;
    int* p = tp;
    for (int c = 0; c < P.L2; ++c) { a[c] = 1; b[c] = 1; pa[c] = 1; pb[c] = 1; }
    const int r0 = dir == 0 ? 0 : P.L1 - 1;
    const int step = dir == 0 ? 1 : -1;
    for (int rr = r0;; rr += step) {
      if (rr == r) {
        for (int c = 0; c < P.L2; ++c) { pa[c] = a[c]; pb[c] = b[c]; }
      }
      for (int c = 0; c < P.L2; ++c) {
        int Dl, Du, Dr, Dd;
        leg_dims(P, rr, c, Dl, Du, Dr, Dd);
        a[c] *= Dl;
        b[c] *= Dr;
        p[c] = dir == 0 ? Dd : Du;
      }
      compressed_dims(P.L2, p, a, b, P.chi);
      if (rr == r) {
        for (int c = 0; c < P.L2; ++c) { oa[c] = a[c]; ob[c] = b[c]; }
        break;
      }
    }
    int po = 0;
    for (int i = 0; i < r * P.L2; ++i) po += P.d2 * block_size(P, i / P.L2, i % P.L2);
    bad = 0;
    for (int c = 0; c < P.L2; ++c) {
      poffr[c] = po;
      po += P.d2 * block_size(P, r, c);
      int Dl, Du, Dr, Dd;
      leg_dims(P, r, c, Dl, Du, Dr, Dd);
      if ((dir == 0 ? Dd : Du) != DP) bad = 1;   // rows (x, p) of the QR need p = DP
    }
    if (bad) set_status(status, PEPS_ERR_UNSUPPORTED);
  }
  __syncthreads();
  if (bad) return;
  const double ls_prev = has_prev ? lsb[rp] : 0.0;

  // 1. absorption
  for (int c = 0; c < P.L2; ++c) {
    int Dl, Du, Dr, Dd;
    leg_dims(P, r, c, Dl, Du, Dr, Dd);
    const int i = r * P.L2 + c;
    const double* W = theta + poffr[c] + (size_t)cfg[i] * (Dl * Du * Dr * Dd);
    const double* A = has_prev ? bnd + ((size_t)rp * P.L2 + c) * P.TS : nullptr;
    const int a = has_prev ? pa[c] : 1, b = has_prev ? pb[c] : 1;
    const int qd = has_prev ? (dir == 0 ? Du : Dd) : 1;
    const int pp = dir == 0 ? Dd : Du;
    double* Bc = w.B + (size_t)c * P.BS;
    const int total = a * Dl * pp * b * Dr;
    for (int idx = tid; idx < total; idx += NTC) {
      int rr = idx % Dr, t = idx / Dr;
      int bq = t % b; t /= b;
      int pq = t % pp; t /= pp;
      int l = t % Dl, aa = t / Dl;
      double s = 0.0;
      for (int x = 0; x < qd; ++x) {
        const double Av = A ? A[(aa * qd + x) * b + bq] : 1.0;
        const double Wv = dir == 0 ? W[((l * Du + x) * Dr + rr) * Dd + pq] : W[((l * Du + pq) * Dr + rr) * Dd + x];
        s += Av * Wv;
      }
      Bc[idx] = s;
    }
    if (tid == 0) {
      sa[c] = a * Dl;
      sp[c] = pp;
      sb[c] = b * Dr;
    }
  }
  __syncthreads();

  // 2. QR sweep.  Wave w owns columns 8w..8w+7 and lane l rows 4l..4l+3,
  // so a column lives in one wave: its norm and the trailing-column dot
  // products are wave reductions (DPP + swizzle), and a Householder step
  // needs a single workgroup barrier, after the owner wave has published
  // v and tau (double-buffered) in LDS.
  double av[QR_RPL][QR_CPW];
  double* Rs = bufB;   // zero-padded 64 x 64 copy of R (stride SV_LD)
  const int lane = tid & 63;
  const int wv_id = tid >> 6;
  const int c0 = QR_CPW * wv_id;     // first column of this wave
  const int r0 = QR_RPL * lane;      // first row of this lane
  {
    const int m = sa[0] * sp[0], n = sb[0];
#pragma unroll
    for (int i = 0; i < QR_RPL; ++i)
#pragma unroll
      for (int cc = 0; cc < QR_CPW; ++cc) {
        const int row = r0 + i, cl = c0 + cc;
        av[i][cc] = (row < m && cl < n) ? w.B[row * n + cl] : 0.0;
      }
  }
  for (int c = 0; c < P.L2 - 1; ++c) {
    const int m = sa[c] * sp[c], n = sb[c];
    const int k = m < n ? m : n;
    // ---- factorisation ----
    for (int j = 0; j < k; ++j) {
      const int bf = j & 1;
      const int cj = j % QR_CPW;               // column of j inside its wave
      if (wv_id == j / QR_CPW) {               // owner wave of column j
        double x[QR_RPL];
#pragma unroll
        for (int i = 0; i < QR_RPL; ++i) {
          double t = 0.0;
#pragma unroll
          for (int cc = 0; cc < QR_CPW; ++cc) t = cc == cj ? av[i][cc] : t;
          x[i] = t;
        }
        double ps = 0.0, aj = 0.0;
#pragma unroll
        for (int i = 0; i < QR_RPL; ++i) {
          const int row = r0 + i;
          ps += row > j ? x[i] * x[i] : 0.0;
          aj += row == j ? x[i] : 0.0;
        }
        const double sigma2 = wave_sum(ps);
        const double alpha = wave_sum(aj);
        double tau = 0.0, scale = 0.0, beta = alpha;
        if (sigma2 > 0.0) {
          const double nrm = sqrt(alpha * alpha + sigma2);
          beta = alpha >= 0.0 ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
#pragma unroll
        for (int i = 0; i < QR_RPL; ++i) {
          const int row = r0 + i;
          const double v = row > j ? x[i] * scale : (row == j ? 1.0 : 0.0);
          qv[bf][row] = v;
          const double nx = row > j ? v : (row == j ? beta : x[i]);
#pragma unroll
          for (int cc = 0; cc < QR_CPW; ++cc) av[i][cc] = cc == cj ? nx : av[i][cc];
        }
        if (lane == 0) { qtau[bf] = tau; taus[j] = tau; }
      }
      __syncthreads();
      const double tau = qtau[bf];
      if (tau != 0.0 && c0 + QR_CPW > j + 1 && c0 < n) {
        double v[QR_RPL];
#pragma unroll
        for (int i = 0; i < QR_RPL; ++i) v[i] = qv[bf][r0 + i];
#pragma unroll
        for (int cc = 0; cc < QR_CPW; ++cc) {
          const int cl = c0 + cc;
          if (cl > j && cl < n) {        // uniform over the wave
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < QR_RPL; ++i) s += v[i] * av[i][cc];
            const double tw = tau * wave_sum(s);
#pragma unroll
            for (int i = 0; i < QR_RPL; ++i) av[i][cc] -= tw * v[i];
          }
        }
      }
    }
    __syncthreads();
    // zero-padded copy of R (rows >= k and below the diagonal are 0); rows < 64
    if (lane < QR_COLS / QR_RPL) {
#pragma unroll
      for (int i = 0; i < QR_RPL; ++i)
#pragma unroll
        for (int cc = 0; cc < QR_CPW; ++cc) {
          const int x = r0 + i, cl = c0 + cc;
          Rs[x * SV_LD + cl] = (x < k && x <= cl && cl < n) ? av[i][cc] : 0.0;
        }
    }
    // ---- explicit thin Q (m x k) by backward accumulation ----
    for (int j = k - 1; j >= 0; --j) {
      const int bf = j & 1;
      const int cj = j % QR_CPW;
      const double tau = taus[j];
      const bool own = wv_id == j / QR_CPW;
      if (own) {
#pragma unroll
        for (int i = 0; i < QR_RPL; ++i) {
          const int row = r0 + i;
          double t = 0.0;
#pragma unroll
          for (int cc = 0; cc < QR_CPW; ++cc) t = cc == cj ? av[i][cc] : t;
          qv[bf][row] = row > j ? t : (row == j ? 1.0 : 0.0);
        }
      }
      __syncthreads();
      if (tau != 0.0 && c0 + QR_CPW > j + 1 && c0 < k) {
        double v[QR_RPL];
#pragma unroll
        for (int i = 0; i < QR_RPL; ++i) v[i] = qv[bf][r0 + i];
#pragma unroll
        for (int cc = 0; cc < QR_CPW; ++cc) {
          const int cl = c0 + cc;
          if (cl > j && cl < k) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < QR_RPL; ++i) s += v[i] * av[i][cc];
            const double tw = tau * wave_sum(s);
#pragma unroll
            for (int i = 0; i < QR_RPL; ++i) av[i][cc] -= tw * v[i];
          }
        }
      }
      if (own) {
#pragma unroll
        for (int i = 0; i < QR_RPL; ++i) {
          const int row = r0 + i;
#pragma unroll
          for (int cc = 0; cc < QR_CPW; ++cc)
            if (cc == cj) av[i][cc] = row < j ? 0.0 : (row == j ? 1.0 - tau : -tau * av[i][cc]);
        }
      }
    }
    __syncthreads();
    // Q -> B_c as [m][k]
    double* Bc = w.B + (size_t)c * P.BS;
#pragma unroll
    for (int i = 0; i < QR_RPL; ++i)
#pragma unroll
      for (int cc = 0; cc < QR_CPW; ++cc) {
        const int row = r0 + i, cl = c0 + cc;
        if (row < m && cl < k) Bc[row * k + cl] = av[i][cc];
      }
    // next matrix: (R B_{c+1}) with rows (x, p), p fastest; B_{c+1}[j][p][b].
    // Lane l holds rows 4l..4l+3, i.e. x = (4l + i) / DP, p = (4l + i) % DP.
    const int pn = sp[c + 1], nn = sb[c + 1];
    const double* Bn = w.B + (size_t)(c + 1) * P.BS;
#pragma unroll
    for (int i = 0; i < QR_RPL; ++i)
#pragma unroll
      for (int cc = 0; cc < QR_CPW; ++cc) av[i][cc] = 0.0;
    // B_{c+1} is staged through LDS (bufA, free during the QR sweep) in
    // chunks of PJ rows, so each wave reads its wave-uniform operands with
    // broadcast LDS loads instead of one global load per operand.
    {
      constexpr int PJ = 16;
      const int rowlen = pn * nn;            // <= DP * 64
      double* stage = bufA;                  // PJ * rowlen <= 16 * 256 doubles
      for (int j0 = 0; j0 < n; j0 += PJ) {
        const int jn = n - j0 < PJ ? n - j0 : PJ;
        for (int idx = tid; idx < jn * rowlen; idx += NTC) stage[idx] = Bn[(size_t)j0 * rowlen + idx];
        __syncthreads();
        if (c0 < nn) {
          for (int jj = 0; jj < jn; ++jj) {
            double rx[QR_RPL];
#pragma unroll
            for (int i = 0; i < QR_RPL; ++i) {
              const int x = (r0 + i) / DP;
              rx[i] = x < QR_COLS ? Rs[x * SV_LD + j0 + jj] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < QR_RPL; ++i) {
              const int pq = i % DP;             // r0 is a multiple of QR_RPL, and DP divides QR_RPL
              const double* brow = stage + (jj * pn + pq) * nn + c0;
#pragma unroll
              for (int cc = 0; cc < QR_CPW; ++cc) av[i][cc] += rx[i] * (c0 + cc < nn ? brow[cc] : 0.0);
            }
          }
        }
        __syncthreads();
      }
    }
    if (tid == 0) {
      sb[c] = k;
      sa[c + 1] = k;
    }
    __syncthreads();
  }
  {
    const int c = P.L2 - 1;
    const int m = sa[c] * sp[c], n = sb[c];
    double* Bc = w.B + (size_t)c * P.BS;
#pragma unroll
    for (int i = 0; i < QR_RPL; ++i)
#pragma unroll
      for (int cc = 0; cc < QR_CPW; ++cc) {
        const int row = r0 + i, cl = c0 + cc;
        if (row < m && cl < n) Bc[row * n + cl] = av[i][cc];
      }
    __syncthreads();
  }

  // 3. truncation sweep
  double* G = bufA;
  double* V = bufB;
  for (int c = P.L2 - 1; c >= 1; --c) {
    const int a = sa[c], nb = sp[c] * sb[c];
    const bool tr = a <= nb;
    const int mg = tr ? nb : a, ng = tr ? a : nb;
    const int k2 = P.chi < ng ? P.chi : ng;
    const double* M = w.B + (size_t)c * P.BS;
    double* Vt = outT + (size_t)c * P.TS;
    if (k2 == nb) {
      // No truncation and M has no more columns than rows: the identity is
      // an orthonormal right factor, so A_c <- 1 and U S = M (same state as
      // an SVD, other gauge).
      for (int idx = tid; idx < nb * nb; idx += NTC) Vt[idx] = (idx / nb == idx % nb) ? 1.0 : 0.0;
      for (int idx = tid; idx < a * nb; idx += NTC) {
        const int i = idx / nb, t = idx % nb;
        V[i * SV_LD + t] = M[idx];
      }
      __syncthreads();
    } else {
    for (int idx = tid; idx < mg * ng; idx += NTC) {
      const int j = idx / mg, i = idx % mg;
      G[j * SV_LD + i] = tr ? M[j * nb + i] : M[i * nb + j];
    }
    if (!tr)
      for (int idx = tid; idx < ng * ng; idx += NTC) {
        const int j = idx / ng, i = idx % ng;
        V[j * SV_LD + i] = (i == j) ? 1.0 : 0.0;
      }
    __syncthreads();
    jacobi64(G, mg, ng, tr ? nullptr : V, flags);
    for (int j = tid; j < ng; j += NTC) {
      double s = 0.0;
      for (int i = 0; i < mg; ++i) s += G[j * SV_LD + i] * G[j * SV_LD + i];
      sig[j] = sqrt(s);
    }
    __syncthreads();
    for (int j = tid; j < ng; j += NTC) {
      int rk = 0;
      for (int t = 0; t < ng; ++t)
        if (sig[t] > sig[j] || (sig[t] == sig[j] && t < j)) ++rk;
      rnk[j] = rk;
    }
    __syncthreads();
    if (tr) {
      // V_k^T rows: normalised columns of G (in place), then U S = M V_k into bufB
      for (int idx = tid; idx < ng * mg; idx += NTC) {
        const int j = idx / mg, e = idx % mg;
        const int rq = rnk[j];
        if (rq < k2) {
          const double v = sig[j] > 0.0 ? G[j * SV_LD + e] / sig[j] : 0.0;
          G[j * SV_LD + e] = v;
          Vt[rq * nb + e] = v;
        }
      }
      __syncthreads();
      for (int idx = tid; idx < a * ng; idx += NTC) {
        const int i = idx / ng, j = idx % ng;
        const int rq = rnk[j];
        if (rq < k2) {
          double s = 0.0;
          for (int e = 0; e < nb; ++e) s += M[i * nb + e] * G[j * SV_LD + e];
          V[i * SV_LD + rq] = s;
        }
      }
    } else {
      for (int idx = tid; idx < ng * ng; idx += NTC) {
        const int j = idx / ng, e = idx % ng;
        const int rq = rnk[j];
        if (rq < k2) Vt[rq * nb + e] = V[j * SV_LD + e];
      }
      __syncthreads();
      for (int idx = tid; idx < a * ng; idx += NTC) {
        const int i = idx / ng, j = idx % ng;
        const int rq = rnk[j];
        if (rq < k2) V[i * SV_LD + rq] = G[j * SV_LD + i];   // U S column, after V was consumed
      }
    }
    __syncthreads();
    }
    // B_{c-1} (m2 x a) <- B_{c-1} (U S) (a x k2), through LDS (G is free)
    const int m2 = sa[c - 1] * sp[c - 1];
    double* Bp = w.B + (size_t)(c - 1) * P.BS;
    for (int idx = tid; idx < m2 * k2; idx += NTC) {
      const int i = idx / k2, t = idx % k2;
      double s = 0.0;
      for (int j = 0; j < a; ++j) s += Bp[i * a + j] * V[j * SV_LD + t];
      G[idx] = s;
    }
    __syncthreads();
    for (int idx = tid; idx < m2 * k2; idx += NTC) Bp[idx] = G[idx];
    if (tid == 0) {
      sb[c - 1] = k2;
      sa[c] = k2;
    }
    __syncthreads();
  }

  // 4. normalise site 0, accumulate the log-scale
  const int tot0 = sa[0] * sp[0] * sb[0];
  double pt = 0.0;
  for (int idx = tid; idx < tot0; idx += NTC) pt += w.B[idx] * w.B[idx];
  const double nrm = sqrt(block_sum512(pt, red));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int idx = tid; idx < tot0; idx += NTC) outT[idx] = w.B[idx] * inv;
  if (tid == 0) {
    lsb[r] = nrm > 0.0 ? ls_prev + log(nrm) : -INFINITY;
    for (int c = 0; c < P.L2; ++c)
      if (sa[c] != oa[c] || sb[c] != ob[c]) set_status(status, PEPS_ERR_UNSUPPORTED);
  }
  // 5. FP32 copy of the row for the mixed-precision strips
  if (P.mixed) {
    __syncthreads();
    float* o32 = (float*)(ws + (size_t)ch * P.chain_stride + (dir == 0 ? P.off_top32 : P.off_bot32)) +
                 (size_t)r * P.L2 * P.TS;
    for (int idx = tid; idx < P.L2 * P.TS; idx += NTC) o32[idx] = (float)outT[idx];
  }
}

bool compress2_supported(const Prob& P) {
  const int cd = P.chi * P.D;
  if (!(P.D == 1 || P.D == 2 || P.D == 4)) return false;
  if (cd > SV_MAX) return false;                 // truncation matrices and QR columns
  if (cd * P.D > QR_ROWS_MAX) return false;      // QR rows
  if (P.L2 > MAX_L) return false;
  return true;
}

hipError_t launch_compress2(const Prob& P, int n, int dir, int r, const double* theta, const uint8_t* configs,
                            double* ws, int32_t* status, hipStream_t st) {
  switch (P.D) {
    case 1: hipLaunchKernelGGL(k_compress2<1>, dim3(n), dim3(NTC), 0, st, P, dir, r, theta, configs, ws, status); break;
    case 2: hipLaunchKernelGGL(k_compress2<2>, dim3(n), dim3(NTC), 0, st, P, dir, r, theta, configs, ws, status); break;
    default: hipLaunchKernelGGL(k_compress2<4>, dim3(n), dim3(NTC), 0, st, P, dir, r, theta, configs, ws, status); break;
  }
  return hipGetLastError();
}

}  // namespace peps
