// Boundary-row compression, register-resident version (one workgroup of 512
// threads per chain).
//
//   1. absorb the row into the boundary: B_c[(a,l)][p][(b,r)];
//   2. left-to-right thin Householder QR with the matrix in registers (32
//      groups of 16 lanes, group g owning columns 2g and 2g+1 and lane t
//      rows 16t..16t+15), one workgroup barrier per reflector; the reflectors
//      (not Q) are stored, R is kept in LDS and R B_{c+1} is formed straight
//      into the registers of the next step (rows (x, p) of the next matrix,
//      p fastest);
//   3. right-to-left truncation by one-sided Jacobi in LDS: G = M^T when M is
//      wide or square (no accumulation; U S = M V_k afterwards), G = M with an
//      accumulated V when M is tall; the left factor U S is carried into the
//      next site by applying that site's reflectors to it (Q (U S) without
//      forming Q), each wave on its own columns with no workgroup barrier;
//   4. normalisation and log-scale.
// Supported shapes: matrices up to 256 x 64 in the QR sweep, 64 x 64 in the
// truncation (chi * D <= 64), physical dimension D in {1, 2, 4}.
#include <math.h>

#include <type_traits>

#include "peps_common.hpp"
#include "peps_dpp.hpp"
#include "peps_kernels.hpp"

namespace peps {

namespace {

constexpr int NTC = 512;        // threads per workgroup (8 waves)
constexpr int QL = 16;          // QR rows per lane (16 lanes x 16 = 256 rows)
constexpr int QR_ROWS_MAX = 256;
static_assert(QL % 4 == 0, "rows per lane must be a multiple of every supported D");
constexpr int QR_COLS = 64;     // max columns
constexpr int SV_MAX = 64;      // max truncation matrix dimension
constexpr int SV_LD = SV_MAX + 1;
#ifndef PEPS_JL
#define PEPS_JL 16
#endif
constexpr int JL = PEPS_JL;     // lanes per Jacobi pair
constexpr int JR = SV_MAX / JL; // rows per lane
constexpr int JAC_MAX_SWEEPS_V2 = 40;
constexpr double JAC_TOL = 2.0e-15;     // rotate while |g_ij| > tol sqrt(g_ii g_jj)
constexpr double JAC_CONV = 1.0e-8;     // a sweep whose rotations all stay below this is the last:
                                        // convergence is quadratic, so the next would be below 1e-16

struct ChainPtrs {
  double *top, *lstop, *bot, *lsbot, *B, *tmp, *tau;
};

__device__ inline ChainPtrs chain_ptrs(const Prob& P, double* ws, int ch) {
  double* base = ws + (size_t)ch * P.chain_stride;
  ChainPtrs w;
  w.top = base + P.off_top;
  w.lstop = base + P.off_lstop;
  w.bot = base + P.off_bot;
  w.lsbot = base + P.off_lsbot;
  w.B = base + P.off_B;
  w.tmp = base + P.off_tmp;
  w.tau = base + P.off_tau;
  return w;
}

// One absorbed site B_c[(x, p)][(b, r)] = sum_u A[a][u][b] W[l][u][r][p]
// (top; for the bottom boundary the roles of the vertical legs swap), with
// x = (a, l).  A is the previous boundary tensor of the column (none for the
// first row: a = b = 1, A = 1), W the configuration's slice of the site.
struct Absorb {
  const double* A;
  const double* W;
  int b, qd, pp, Dl, Du, Dr, Dd, dir;
  __device__ inline double at(int x, int p, int col) const {
    const int aa = x / Dl, l = x % Dl, bq = col / Dr, rr = col % Dr;
    double s = 0.0;
    for (int u = 0; u < qd; ++u) {
      const double Av = A ? A[(aa * qd + u) * b + bq] : 1.0;
      const double Wv = dir == 0 ? W[((l * Du + u) * Dr + rr) * Dd + p] : W[((l * Du + p) * Dr + rr) * Dd + u];
      s += Av * Wv;
    }
    return s;
  }
};

__device__ inline Absorb absorb_site(const Prob& P, int dir, int r, int c, const double* theta, const uint8_t* cfg,
                                     const double* bnd, int rp, bool has_prev, const int* poffr, const int* pa,
                                     const int* pb) {
  Absorb ab;
  leg_dims(P, r, c, ab.Dl, ab.Du, ab.Dr, ab.Dd);
  ab.W = theta + poffr[c] + (size_t)digit_at(P, cfg, r * P.L2 + c) * (ab.Dl * ab.Du * ab.Dr * ab.Dd);
  ab.A = has_prev ? bnd + ((size_t)rp * P.L2 + c) * P.TS : nullptr;
  ab.b = has_prev ? pb[c] : 1;
  ab.qd = has_prev ? (dir == 0 ? ab.Du : ab.Dd) : 1;
  ab.pp = dir == 0 ? ab.Dd : ab.Du;
  ab.dir = dir;
  (void)pa;
  return ab;
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
__device__ inline double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r;
}
__device__ inline double rcp_nr1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ inline double sqrt1p_sq1(double a) {
  const double y = fma(a, a, 1.0);
  double r = __builtin_amdgcn_rsq(y);
  r = r * fma(-0.5 * y * r, r, 1.5);
  return y * r;
}

// Lane exchange inside one 16-lane DPP row, for a double.  Every control
// used here reads a lane of the same row, so no lane is masked or out of
// bounds and no old value is needed.
// Q X for the thin Q = H_0 H_1 ... H_{k-1} of one QR step, with
// H_j = 1 - tau_j v_j v_j^T, the v_j stored column-major (m rows each, unit
// entry and zeros above it included), and X = [US; 0] of m x nx with US the
// first k rows (stride ldu).  Wave w takes columns w, w + 8, ... (NCW per
// wave), lane l rows 4l..4l+3; the waves never synchronise.  The result is
// written row-major (m x nx) to out.
template <int NCW>
__device__ inline void apply_q(const double* __restrict__ vs, const double* __restrict__ taus, int m, int k,
                               const double* US, int ldu, int nx, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = 4 * lane;
  double x[4][NCW];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < NCW; ++q) {
      const int row = r0 + i, col = wave + 8 * q;
      x[i][q] = (row < k && col < nx) ? US[row * ldu + col] : 0.0;
    }
  if (wave < nx && k > 0) {
    // reflector j+1's data is consumed while reflector j's is in flight
    double vn[4], taun = taus[k - 1];
#pragma unroll
    for (int i = 0; i < 4; ++i) vn[i] = r0 + i < m ? vs[(size_t)(k - 1) * m + r0 + i] : 0.0;
    for (int j = k - 1; j >= 0; --j) {
      const double tau = taun;
      double v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = vn[i];
      if (j > 0) {
        taun = taus[j - 1];
#pragma unroll
        for (int i = 0; i < 4; ++i) vn[i] = r0 + i < m ? vs[(size_t)(j - 1) * m + r0 + i] : 0.0;
      }
      if (tau == 0.0) continue;   // uniform: every lane reads the same tau
      double sd[NCW];
#pragma unroll
      for (int q = 0; q < NCW; ++q) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) t += v[i] * x[i][q];
        sd[q] = t;
      }
      wave_sum_n<NCW>(sd);
#pragma unroll
      for (int q = 0; q < NCW; ++q) {
        const double tw = tau * sd[q];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i][q] -= tw * v[i];
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < NCW; ++q) {
        const int row = r0 + i, col = wave + 8 * q;
        if (row < m && col < nx) out[row * nx + col] = x[i][q];
      }
  }
}

// Sum over the JL lanes of a Jacobi pair (aligned groups inside a DPP
// row), identical bits on every lane of the group.
__device__ inline double pair_sum(double v) {
  v += dpp_f64<0xB1>(v);                       // quad_perm [1,0,3,2]
  if (JL >= 4) v += dpp_f64<0x4E>(v);          // quad_perm [2,3,0,1]
  if (JL >= 8) v += dpp_f64<0x141>(v);         // row_half_mirror
  if (JL >= 16) v += dpp_f64<0x140>(v);        // row_mirror
  return v;
}

// One-sided Jacobi on G (mg x ng <= 64 x 64, column-major, stride SV_LD),
// optionally accumulating V (ng x ng, column-major, stride SV_LD).  Rows
// mg..63 of G and ng..63 of V must hold zeros: every lane then works on its
// four rows without bounds tests (zero rows change no dot product).
__device__ void jacobi64(double* G, int mg, int ng, double* V, int* flags) {
  const int tid = threadIdx.x;
  if (ng < 2) return;
  const int ne = ng + (ng & 1);
  const int npairs = ne / 2;
  const int grp = tid / JL, lane = tid % JL;
  if (tid == 0) { flags[0] = 0; flags[1] = 0; }
  __syncthreads();
  // round-robin (circle) order: in round rnd group 0 pairs (rnd, ne-1) and
  // group g > 0 pairs ((rnd + g) mod (ne-1), (rnd - g) mod (ne-1)); both
  // indices advance by one per round.
  const bool active = grp < npairs;
  for (int sweep = 0; sweep < JAC_MAX_SWEEPS_V2; ++sweep) {
    const int fl = sweep & 1;
    int pi = grp == 0 ? 0 : grp % (ne - 1);
    int pj = grp == 0 ? ne - 1 : (ne - 1 - grp) % (ne - 1);
    for (int rnd = 0; rnd < ne - 1; ++rnd) {
      const int ci = pi < pj ? pi : pj, cj = pi < pj ? pj : pi;
      if (active && cj < ng) {                  // uniform over the group
        double x[JR], y[JR];
        double al = 0.0, be = 0.0, ga = 0.0;
        const double* gi = G + ci * SV_LD;
        const double* gj = G + cj * SV_LD;
#pragma unroll
        for (int t = 0; t < JR; ++t) {
          const int i = lane + JL * t;
          x[t] = gi[i];
          y[t] = gj[i];
          al += x[t] * x[t];
          be += y[t] * y[t];
          ga += x[t] * y[t];
        }
        al = pair_sum(al);
        be = pair_sum(be);
        ga = pair_sum(ga);
        if (ga != 0.0 && ga * ga > (JAC_TOL * JAC_TOL) * (al * be)) {
          // Rotation (Rutishauser's angle, |theta| <= pi/4) from the double
          // angle: with d = be - al, e = 2 ga, r = |(d, e)|, cos 2theta =
          // |d| / r and sin 2theta = sign(d) e / r, so (c, s) is parallel to
          // ((1 + cos 2theta) / 2, sin 2theta / 2).  That vector is
          // normalised by a full-precision 1/sqrt, so c^2 + s^2 = 1 to
          // rounding whatever the error of 1/r, which only perturbs the
          // angle (the next sweep corrects it): 1/r is the hardware
          // estimate, unrefined.  Out of range of d^2 + e^2:
          // the same angle through the cotangent.
          const double d = be - al, e = 2.0 * ga;
          const double r2 = fma(d, d, e * e);
          double c, s;
          if (r2 < 1.0e300 && r2 > 1.0e-300) {
            const double u = __builtin_amdgcn_rsq(r2);   // sets the angle only
            const double h = fma(0.5 * fabs(d), u, 0.5);
            const double q = (d >= 0.0 ? 0.5 : -0.5) * e * u;
            const double w = rsqrt_nr(fma(h, h, q * q));
            c = h * w;
            s = q * w;
          } else {
            const double zeta = (be - al) * rcp_nr1(2.0 * ga);
            const double az = fabs(zeta);
            const double root = az < 1.0e150 ? sqrt1p_sq1(az) : az;
            const double t = copysign(rcp_nr1(az + root), zeta);
            c = rsqrt_nr(fma(t, t, 1.0));
            s = c * t;
          }
          double* gwi = G + ci * SV_LD;
          double* gwj = G + cj * SV_LD;
#pragma unroll
          for (int tt = 0; tt < JR; ++tt) {
            const int i = lane + JL * tt;
            gwi[i] = c * x[tt] - s * y[tt];
            gwj[i] = s * x[tt] + c * y[tt];
          }
          if (V) {
            double* vi = V + ci * SV_LD;
            double* vj = V + cj * SV_LD;
#pragma unroll
            for (int tt = 0; tt < JR; ++tt) {
              const int i = lane + JL * tt;
              const double a = vi[i], b = vj[i];
              vi[i] = c * a - s * b;
              vj[i] = s * a + c * b;
            }
          }
          if (lane == 0 && ga * ga > (JAC_CONV * JAC_CONV) * (al * be)) flags[fl] = 1;
        }
      }
      __syncthreads();
      if (grp != 0) pi = pi + 1 == ne - 1 ? 0 : pi + 1;
      else pi = pi + 1;
      pj = (grp != 0 && pj + 1 == ne - 1) ? 0 : (grp != 0 ? pj + 1 : pj);
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
  __shared__ int perm[SV_MAX];

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

  // 1. absorption: only the dims here; each site's absorbed tensor is formed
  // where it is consumed (the first QR matrix, and the staged rows of
  // R B_{c+1}), never stored
  if (tid == 0)
    for (int c = 0; c < P.L2; ++c) {
      int Dl, Du, Dr, Dd;
      leg_dims(P, r, c, Dl, Du, Dr, Dd);
      sa[c] = (has_prev ? pa[c] : 1) * Dl;
      sp[c] = dir == 0 ? Dd : Du;
      sb[c] = (has_prev ? pb[c] : 1) * Dr;
    }
  __syncthreads();

  // 2. QR sweep.  The workgroup is 32 groups of 16 lanes (one DPP row
  // each); group g owns columns 2g, 2g+1 and lane t of the group rows
  // 16t..16t+15.  A column lives inside one DPP row, so its norm and the
  // trailing dot products are 16-lane DPP reductions, and a Householder step
  // needs a single workgroup barrier, after the owner group has published v
  // and tau (double-buffered) in LDS.
  double av[QL][2];
  double* Rs = bufB;   // zero-padded 64 x 64 copy of R (stride SV_LD)
  const int grp = tid >> 4;
  const int gl = tid & 15;
  const int c0 = 2 * grp;      // first column of this group
  const int r0 = QL * gl;      // first row of this lane
  {
    const int m = sa[0] * sp[0], n = sb[0];
    const Absorb ab = absorb_site(P, dir, r, 0, theta, cfg, bnd, rp, has_prev, poffr, pa, pb);
#pragma unroll
    for (int i = 0; i < QL; ++i)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int row = r0 + i, cl = c0 + q;
        av[i][q] = (row < m && cl < n) ? ab.at(row / ab.pp, row % ab.pp, cl) : 0.0;
      }
  }
  for (int c = 0; c < P.L2 - 1; ++c) {
    const int m = sa[c] * sp[c], n = sb[c];
    const int k = m < n ? m : n;
    // ---- factorisation ----
    // One Householder step for column j, which is column COL (0 or 1) of its
    // owner group; COL is a compile-time index into the register slice.
    auto qr_step = [&](int j, auto colc) {
      constexpr int COL = decltype(colc)::value;
      const int bf = j & 1;
      if (grp == (j >> 1)) {                  // owner group of column j
        const int dj = j - r0;                // row r0 + i is below the diagonal when i > dj
        // four interleaved partial sums: dependency chains of QL / 4
        double s2p[4] = {0.0, 0.0, 0.0, 0.0}, alp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < QL; ++i) {
          const double xi = av[i][COL];
          s2p[i & 3] += i > dj ? xi * xi : 0.0;
          alp[i & 3] += i == dj ? xi : 0.0;
        }
        double s2[2] = {(s2p[0] + s2p[1]) + (s2p[2] + s2p[3]), (alp[0] + alp[1]) + (alp[2] + alp[3])};
        row16_sum_n<2>(s2);
        const double sigma2 = s2[0], alpha = s2[1];
        double tau = 0.0, scale = 0.0, beta = alpha;
        if (sigma2 > 0.0) {
          const double nrm = sqrt(alpha * alpha + sigma2);
          beta = alpha >= 0.0 ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
#pragma unroll
        for (int i = 0; i < QL; ++i) {
          const double xi = av[i][COL];
          const double v = i > dj ? xi * scale : (i == dj ? 1.0 : 0.0);
          qv[bf][r0 + i] = v;
          av[i][COL] = i > dj ? v : (i == dj ? beta : xi);
        }
        if (gl == 0) { qtau[bf] = tau; taus[j] = tau; }
      }
      __syncthreads();
      const double tau = qtau[bf];
      if (tau != 0.0 && c0 + 1 > j && c0 < n) {   // the group has a column right of j
        // v is streamed from LDS twice (dots, then update) rather than held in
        // 16 more register pairs next to the 32 of the matrix slice
        // two interleaved partial sums per column: chains of QL / 2
        double sp0[2] = {0.0, 0.0}, sp1[2] = {0.0, 0.0};
#pragma unroll
        for (int i = 0; i < QL; ++i) {
          const double vi = qv[bf][r0 + i];
          sp0[i & 1] += vi * av[i][0];
          sp1[i & 1] += vi * av[i][1];
        }
        double sd[2] = {sp0[0] + sp0[1], sp1[0] + sp1[1]};
        row16_sum_n<2>(sd);
        const double tw0 = (c0 > j && c0 < n) ? tau * sd[0] : 0.0;
        const double tw1 = (c0 + 1 > j && c0 + 1 < n) ? tau * sd[1] : 0.0;
        asm volatile("" ::: "memory");   // compiler-only fence: reload v below
#pragma unroll
        for (int i = 0; i < QL; ++i) {
          const double vi = qv[bf][r0 + i];
          av[i][0] -= tw0 * vi;
          av[i][1] -= tw1 * vi;
        }
      }
    };
    for (int j = 0; j < k; j += 2) {
      qr_step(j, std::integral_constant<int, 0>());
      if (j + 1 < k) qr_step(j + 1, std::integral_constant<int, 1>());
    }
    __syncthreads();
    // zero-padded copy of R (rows >= k and below the diagonal are 0); rows < 64
    if (r0 < QR_COLS) {
#pragma unroll
      for (int i = 0; i < QL; ++i)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int x = r0 + i, cl = c0 + q;
          Rs[x * SV_LD + cl] = (x < k && x <= cl && cl < n) ? av[i][q] : 0.0;
        }
    }
    // ---- reflectors v_j (column-major, unit entry and zeros above it
    // included) into B_c, their scalars into tau[c] ----
    {
      double* Vs = w.B + (size_t)c * P.BS;
#pragma unroll
      for (int i = 0; i < QL; ++i)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int row = r0 + i, cl = c0 + q;
          if (row < m && cl < k) Vs[(size_t)cl * m + row] = row > cl ? av[i][q] : (row == cl ? 1.0 : 0.0);
        }
      for (int j = tid; j < k; j += NTC) w.tau[c * (P.chi * P.D) + j] = taus[j];
    }
    // next matrix: (R B_{c+1}) with rows (x, p), p fastest; B_{c+1}[y][p][b].
    // Lane t holds rows 16t..16t+15, i.e. x = (16t + i) / DP, p = i % DP.
    const int pn = sp[c + 1], nn = sb[c + 1];
    const Absorb abn = absorb_site(P, dir, r, c + 1, theta, cfg, bnd, rp, has_prev, poffr, pa, pb);
#pragma unroll
    for (int i = 0; i < QL; ++i) {
      av[i][0] = 0.0;
      av[i][1] = 0.0;
    }
    // B_{c+1} is staged through LDS (bufA, free during the QR sweep) in
    // chunks of PJ rows.
    {
      constexpr int PJ = 16;
      const int rowlen = pn * nn;            // <= DP * 64
      double* stage = bufA;                  // PJ * rowlen <= 16 * 256 doubles
      const int x0 = r0 / DP;
      for (int j0 = 0; j0 < n; j0 += PJ) {
        const int jn = n - j0 < PJ ? n - j0 : PJ;
        for (int idx = tid; idx < jn * rowlen; idx += NTC) {
          const int jj = idx / rowlen, rem = idx % rowlen;
          stage[idx] = abn.at(j0 + jj, rem / nn, rem % nn);
        }
        __syncthreads();
        if (c0 < nn) {
          for (int jj = 0; jj < jn; ++jj) {
            double rx[QL / DP];
#pragma unroll
            for (int xi = 0; xi < QL / DP; ++xi) {
              const int x = x0 + xi;
              rx[xi] = x < QR_COLS ? Rs[x * SV_LD + j0 + jj] : 0.0;
            }
#pragma unroll
            for (int pq = 0; pq < DP; ++pq) {
              const double* brow = stage + (jj * pn + pq) * nn + c0;
              const double b0 = brow[0];
              const double b1 = c0 + 1 < nn ? brow[1] : 0.0;
#pragma unroll
              for (int xi = 0; xi < QL / DP; ++xi) {
                av[xi * DP + pq][0] += rx[xi] * b0;
                av[xi * DP + pq][1] += rx[xi] * b1;
              }
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
    for (int i = 0; i < QL; ++i)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int row = r0 + i, cl = c0 + q;
        if (row < m && cl < n) Bc[row * n + cl] = av[i][q];
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
    // the last site's matrix is dense in B after the QR sweep; every other
    // site's is the product left in tmp by the previous step
    const double* M = c == P.L2 - 1 ? w.B + (size_t)c * P.BS : w.tmp;
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
    for (int idx = tid; idx < SV_MAX * ng; idx += NTC) {
      const int j = idx / SV_MAX, i = idx % SV_MAX;
      G[j * SV_LD + i] = i >= mg ? 0.0 : (tr ? M[j * nb + i] : M[i * nb + j]);
    }
    if (!tr)
      for (int idx = tid; idx < SV_MAX * ng; idx += NTC) {
        const int j = idx / SV_MAX, i = idx % SV_MAX;
        V[j * SV_LD + i] = (i == j) ? 1.0 : 0.0;
      }
    __syncthreads();
    jacobi64(G, mg, ng, tr ? nullptr : V, flags);
    {
      // column norms: 16 lanes per column (rows zero-padded to 64)
      const int g16 = tid >> 4, l16 = tid & 15;
      for (int j = g16; j < ng; j += NTC / 16) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < SV_MAX / 16; ++t) {
          const double x = G[j * SV_LD + l16 + 16 * t];
          s += x * x;
        }
        s = row16_sum(s);
        if (l16 == 0) sig[j] = rank_norm(s, status);
      }
    }
    __syncthreads();
    for (int j = tid; j < ng; j += NTC) {
      int rk = 0;
      for (int t = 0; t < ng; ++t)
        if (sig[t] > sig[j] || (sig[t] == sig[j] && t < j)) ++rk;
      rnk[j] = rk;
      perm[rk] = j;
    }
    __syncthreads();
    if (tr) {
      // V_k^T rows: normalised kept columns of G (in place), then U S = M V_k
      for (int idx = tid; idx < k2 * mg; idx += NTC) {
        const int rq = idx / mg, e = idx % mg;
        const int j = perm[rq];
        const double v = sig[j] > 0.0 ? G[j * SV_LD + e] / sig[j] : 0.0;
        G[j * SV_LD + e] = v;
        Vt[rq * nb + e] = v;
      }
      __syncthreads();
      for (int idx = tid; idx < a * k2; idx += NTC) {
        const int i = idx / k2, rq = idx % k2;
        const double* gj = G + perm[rq] * SV_LD;
        const double* mi = M + i * nb;
        double s = 0.0;
        for (int e = 0; e < nb; ++e) s += mi[e] * gj[e];
        V[i * SV_LD + rq] = s;
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
    // A_{c-1} <- Q_{c-1} (U S): the reflectors of QR step c-1 applied to
    // U S (a x k2, in V), written row-major (m2 x k2) to tmp
    {
      const int m2 = sa[c - 1] * sp[c - 1];
      const double* vs = w.B + (size_t)(c - 1) * P.BS;
      const double* tc = w.tau + (size_t)(c - 1) * (P.chi * P.D);
      if (k2 <= 8) apply_q<1>(vs, tc, m2, a, V, SV_LD, k2, w.tmp);
      else if (k2 <= 16) apply_q<2>(vs, tc, m2, a, V, SV_LD, k2, w.tmp);
      else if (k2 <= 32) apply_q<4>(vs, tc, m2, a, V, SV_LD, k2, w.tmp);
      else apply_q<8>(vs, tc, m2, a, V, SV_LD, k2, w.tmp);
    }
    __syncthreads();
    if (tid == 0) {
      sb[c - 1] = k2;
      sa[c] = k2;
    }
    __syncthreads();
  }

  // 4. normalise site 0, accumulate the log-scale
  const int tot0 = sa[0] * sp[0] * sb[0];
  double pt = 0.0;
  for (int idx = tid; idx < tot0; idx += NTC) pt += w.tmp[idx] * w.tmp[idx];
  const double nrm = sqrt(block_sum512(pt, red));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int idx = tid; idx < tot0; idx += NTC) outT[idx] = w.tmp[idx] * inv;
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
