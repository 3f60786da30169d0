// Boundary-row compression for bond dimensions whose QR matrices do not fit
// on chip (chi * D beyond the register kernel, matrices beyond LDS): the
// same two-sweep C_chi as the other compression kernels (boundary-MPS
// contraction with boundary dimension D_c = chi; QR left to right, SVD
// truncation right to left), one 512-thread workgroup per chain, with the
// dense matrices in the chain's workspace:
//   * QR of (a p) x b by blocked Householder (Golub & Van Loan, Alg. 5.2.2,
//     compact WY of Schreiber & Van Loan): panels of up to NBMAX columns
//     factorised in LDS, T factors kept, trailing columns updated one per
//     wave as A - V T^T (V^T A), each column loaded into registers once per
//     panel;
//   * R B_{c+1} as FP64 MFMA tiles;
//   * the truncation by block one-sided Jacobi (Hestenes): per outer sweep
//     the pairs inside every column block, then the pairs between the two
//     blocks of every block pair, each pass in LDS (every column pair once
//     per outer sweep), no rotation accumulation for wide matrices;
//   * Q_{c-1} (U S) applied panel by panel from the reflectors and T of the
//     QR of X_{c-1}: kept from the first sweep, or, in the smaller workspace
//     layout, rebuilt from the stored R_{c-2} and a new absorption of site
//     c-1 (one QR matrix per chain instead of one per site).
#include <math.h>

#include "peps_chain.hpp"
#include "peps_common.hpp"
#include "peps_contract.hpp"
#include "peps_dpp.hpp"
#include "peps_kernels.hpp"
#include "peps_linalg.hpp"

namespace peps {

namespace {

constexpr int NTB = 512;                        // threads per workgroup (two waves per SIMD)
constexpr int NBMAX = 12;                       // widest panel
constexpr int PANEL_DOUBLES = 14 * 1024;        // LDS work array: 112 KB (QR panel, Jacobi blocks, W of Q Y)
constexpr int NWAVE_B = NTB / 64;
// A sweep whose rotations all stay below this relative size is the last
// one.  At the deep truncation chains of this kernel (chi D up to 512, tens
// of truncations per boundary) the reported quantities amplify the
// orthogonality left by the last sweep, so the stop comes one quadratic
// step later than in the small kernel.
constexpr double JAC_CONV_BIG = 1.0e-12;

// Panel width for a QR with m rows (the panel must fit the LDS array).
__host__ __device__ inline int panel_width(int m) {
  int nb = PANEL_DOUBLES / (m > 0 ? m : 1);
  if (nb > NBMAX) nb = NBMAX;
  if (nb < 1) nb = 1;
  return nb;
}

__device__ inline double wave_sum64(double v) { return wave_sum(v); }

// Fixed-order sum over the workgroup (waves, then the NWAVE_B partials).
__device__ inline double block_sum_b(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum64(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < NWAVE_B; ++q) s += red[q];
  __syncthreads();
  return s;
}

// Absorbed site c of row r: element (x = (aa, l), p, col = (bq, rr)) of
// B_c = sum_u A[aa][u][bq] W[l][u][rr][p] (top; the vertical legs swap for the
// bottom boundary).  Written at dst[x * xs + p * ps + col * cs].
__device__ void absorb_site_to(const Prob& P, const Geo& geo, int dir, int r, int c, const double* theta,
                               const uint8_t* cfg, const double* bnd, bool has_prev, int rp, double* dst,
                               int64_t xs, int64_t ps, int64_t cs, int& sa_out, int& sp_out, int& sb_out) {
  int Dl, Du, Dr, Dd;
  leg_dims(P, r, c, Dl, Du, Dr, Dd);
  const int i = r * P.L2 + c;
  const double* W = theta + geo.poff[i] + (size_t)digit_at(P, cfg, i) * (Dl * Du * Dr * Dd);
  const double* A = has_prev ? bnd + ((size_t)rp * P.L2 + c) * P.TS : nullptr;
  const int a = has_prev ? geo.ba[dir][rp][c] : 1;
  const int b = has_prev ? geo.bb[dir][rp][c] : 1;
  const int q = has_prev ? (dir == 0 ? Du : Dd) : 1;
  const int pp = dir == 0 ? Dd : Du;
  const int total = a * Dl * pp * b * Dr;
  for (int idx = threadIdx.x; idx < total; idx += NTB) {
    int rr = idx % Dr, t = idx / Dr;
    const int bq = t % b;
    t /= b;
    const int p = t % pp;
    t /= pp;
    const int l = t % Dl, aa = t / Dl;
    double s = 0.0;
    for (int u = 0; u < q; ++u) {
      const double Av = A ? A[(aa * q + u) * b + bq] : 1.0;
      const double Wv = dir == 0 ? W[((l * Du + u) * Dr + rr) * Dd + p] : W[((l * Du + p) * Dr + rr) * Dd + u];
      s += Av * Wv;
    }
    const int x = aa * Dl + l, col = bq * Dr + rr;
    dst[x * xs + p * ps + col * cs] = s;
  }
  sa_out = a * Dl;
  sp_out = pp;
  sb_out = b * Dr;
}

// Blocked Householder QR of X (m x n, column-major, leading dimension m) in
// place: R on and above the diagonal of the first k = min(m, n) rows, the
// reflectors v_j (unit entry implied) below it, tau_j in taus[j], and the
// upper-triangular T of each panel (Q_panel = I - V T V^T) at
// Tst[j0 * NBMAX ...] (nb x nb, row-major).
__device__ __forceinline__ void qr_blocked(double* X, int m, int n, double* taus, double* Tst, double* panel, double* Tm,
                           double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int k = m < n ? m : n;
  const int NB = panel_width(m);
  for (int j0 = 0; j0 < k; j0 += NB) {
    const int nb = k - j0 < NB ? k - j0 : NB;
    const int rows = m - j0;
    for (int idx = tid; idx < nb * rows; idx += NTB) {
      const int t = idx / rows, i = idx % rows;
      panel[idx] = X[(size_t)(j0 + t) * m + j0 + i];
    }
    __syncthreads();
    // unblocked factorisation of the panel
    for (int t = 0; t < nb; ++t) {
      double* pc = panel + t * rows;
      double part = 0.0;
      for (int i = t + 1 + tid; i < rows; i += NTB) part += pc[i] * pc[i];
      const double sigma2 = block_sum_b(part, red);
      const double alpha = pc[t];
      double tau = 0.0, scale = 0.0, beta = alpha;
      if (sigma2 > 0.0) {
        const double nrm = sqrt(alpha * alpha + sigma2);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      if (tau != 0.0)
        for (int i = t + 1 + tid; i < rows; i += NTB) pc[i] *= scale;
      __syncthreads();
      if (tid == 0) {
        pc[t] = beta;
        taus[j0 + t] = tau;
        Tm[t * NBMAX + t] = tau;
      }
      if (tau != 0.0) {
        for (int u = t + 1 + wave; u < nb; u += NWAVE_B) {
          double* pu = panel + u * rows;
          double s = lane == 0 ? pu[t] : 0.0;
          for (int i = t + 1 + lane; i < rows; i += 64) s += pc[i] * pu[i];
          const double wt = tau * wave_sum64(s);
          if (lane == 0) pu[t] -= wt;
          for (int i = t + 1 + lane; i < rows; i += 64) pu[i] -= pc[i] * wt;
        }
      }
      __syncthreads();
    }
    // T (forward, column-wise): T[0:t, t] = -tau_t T[0:t, 0:t] (V[:, 0:t]^T v_t)
    for (int st = wave; st < nb * nb; st += NWAVE_B) {
      const int s = st / nb, t = st % nb;
      if (s >= t) continue;
      // v_s . v_t over rows >= t (v_t[t] = 1, zero above)
      double d = lane == 0 ? panel[s * rows + t] : 0.0;
      for (int i = t + 1 + lane; i < rows; i += 64) d += panel[s * rows + i] * panel[t * rows + i];
      d = wave_sum64(d);
      if (lane == 0) Tm[s * NBMAX + t] = d;   // dot, replaced by T below
    }
    __syncthreads();
    if (tid == 0) {
      double z[NBMAX];
      for (int t = 1; t < nb; ++t) {
        const double tau = Tm[t * NBMAX + t];
        for (int s = 0; s < t; ++s) z[s] = -tau * Tm[s * NBMAX + t];
        for (int s = 0; s < t; ++s) {
          double v = 0.0;
          for (int q = s; q < t; ++q) v += (q == s ? Tm[s * NBMAX + s] : Tm[s * NBMAX + q]) * z[q];
          Tm[s * NBMAX + t] = v;
        }
      }
      for (int s = 0; s < nb; ++s)
        for (int t = 0; t < nb; ++t) Tst[(size_t)j0 * NBMAX + s * nb + t] = t >= s ? Tm[s * NBMAX + t] : 0.0;
    }
    // panel back to the matrix
    for (int idx = tid; idx < nb * rows; idx += NTB) {
      const int t = idx / rows, i = idx % rows;
      X[(size_t)(j0 + t) * m + j0 + i] = panel[idx];
    }
    __syncthreads();
    // trailing columns: A <- A - V T^T (V^T A), one wave per column; a
    // column of up to 64 RMAX rows is loaded into registers in one batch
    constexpr int RMAX = 24;
    const bool staged = rows <= 64 * RMAX;
    for (int col = j0 + nb + wave; col < n; col += NWAVE_B) {
      double* xc = X + (size_t)col * m + j0;
      double wv[NBMAX];
#pragma unroll
      for (int t = 0; t < NBMAX; ++t) wv[t] = 0.0;
      double xr[RMAX];
      if (staged) {
#pragma unroll
        for (int u = 0; u < RMAX; ++u) {
          const int i = lane + 64 * u;
          xr[u] = i < rows ? xc[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < RMAX; ++u) {
          const int i = lane + 64 * u;
          if (64 * u < rows) {
#pragma unroll
            for (int t = 0; t < NBMAX; ++t)
              if (t < nb) wv[t] += ((i > t && i < rows) ? panel[t * rows + i] : (i == t ? 1.0 : 0.0)) * xr[u];
          }
        }
      } else {
        for (int i = lane; i < rows; i += 64) {
          const double x = xc[i];
#pragma unroll
          for (int t = 0; t < NBMAX; ++t)
            if (t < nb) wv[t] += (i > t ? panel[t * rows + i] : (i == t ? 1.0 : 0.0)) * x;
        }
      }
      // the nb wave sums stage by stage, so that their latencies overlap
#pragma unroll
      for (int t = 0; t < NBMAX; ++t)
        if (t < nb) wv[t] += dpp_f64<0xB1>(wv[t]);
#pragma unroll
      for (int t = 0; t < NBMAX; ++t)
        if (t < nb) wv[t] += dpp_f64<0x4E>(wv[t]);
#pragma unroll
      for (int t = 0; t < NBMAX; ++t)
        if (t < nb) wv[t] += dpp_f64<0x141>(wv[t]);
#pragma unroll
      for (int t = 0; t < NBMAX; ++t)
        if (t < nb) wv[t] += dpp_f64<0x140>(wv[t]);
#pragma unroll
      for (int t = 0; t < NBMAX; ++t)
        if (t < nb) wv[t] = rows_pair_sum(wv[t]);
#pragma unroll
      for (int t = 0; t < NBMAX; ++t)
        if (t < nb) wv[t] = halves_sum(wv[t]);
      double w2[NBMAX];
#pragma unroll
      for (int t = 0; t < NBMAX; ++t) {
        double v = 0.0;
#pragma unroll
        for (int s = 0; s < NBMAX; ++s)
          if (s <= t && s < nb) v += Tm[s * NBMAX + t] * wv[s];
        w2[t] = t < nb ? v : 0.0;
      }
      if (staged) {
#pragma unroll
        for (int u = 0; u < RMAX; ++u) {
          const int i = lane + 64 * u;
          if (64 * u < rows) {
            double x = xr[u];
#pragma unroll
            for (int t = 0; t < NBMAX; ++t)
              if (t < nb) x -= ((i > t && i < rows) ? panel[t * rows + i] : (i == t ? 1.0 : 0.0)) * w2[t];
            if (i < rows) xc[i] = x;
          }
        }
      } else {
        for (int i = lane; i < rows; i += 64) {
          double x = xc[i];
#pragma unroll
          for (int t = 0; t < NBMAX; ++t)
            if (t < nb) x -= (i > t ? panel[t * rows + i] : (i == t ? 1.0 : 0.0)) * w2[t];
          xc[i] = x;
        }
      }
    }
    __syncthreads();
  }
}

// Y <- Q Y for the Q of a blocked QR (X: reflectors, m rows, k of them;
// Tst: panel T factors), Y m x ny row-major with leading dimension ny.
__device__ void apply_q_blocked(const double* X, int m, int k, const double* Tst, double* Y, int ny, double* Wl) {
  const int tid = threadIdx.x;
  const int NB = panel_width(m);
  if (k <= 0) return;
  const int last = ((k - 1) / NB) * NB;
  for (int j0 = last; j0 >= 0; j0 -= NB) {
    const int nb = k - j0 < NB ? k - j0 : NB;
    const int rows = m - j0;
    const double* V = X + (size_t)j0 * m + j0;   // column t at V + t * m
    const double* T = Tst + (size_t)j0 * NBMAX;  // nb x nb
    double* W = Wl;                              // nb x ny
    double* W2 = Wl + NBMAX * ny;                // nb x ny
    double* Wp = Wl + 2 * NBMAX * ny;            // partials [rg][nb][ny]
    // W = V^T Y: thread (rg, q) accumulates the nb sums over rows rg, rg + R,
    // ... (Y loads coalesced along q, V entries shared by the q threads),
    // then the R partials are added in a fixed order
    const int R = NTB / ny > 0 ? NTB / ny : 1;
    const int rg = tid / ny, q0 = tid % ny;
    if (rg < R && tid < R * ny) {
      double wp[NBMAX];
#pragma unroll
      for (int t = 0; t < NBMAX; ++t) wp[t] = 0.0;
#pragma unroll 2
      for (int i = rg; i < rows; i += R) {
        const double y = Y[(size_t)(j0 + i) * ny + q0];
#pragma unroll
        for (int t = 0; t < NBMAX; ++t)
          if (t < nb && t <= i) wp[t] += (i == t ? 1.0 : V[(size_t)t * m + i]) * y;
      }
#pragma unroll
      for (int t = 0; t < NBMAX; ++t)
        if (t < nb) Wp[(rg * nb + t) * ny + q0] = wp[t];
    }
    __syncthreads();
    for (int tq = tid; tq < nb * ny; tq += NTB) {
      const int t = tq / ny, q = tq % ny;
      double s = 0.0;
      for (int g = 0; g < R; ++g) s += Wp[(g * nb + t) * ny + q];
      W[t * ny + q] = s;
    }
    __syncthreads();
    for (int tq = tid; tq < nb * ny; tq += NTB) {
      const int t = tq / ny, q = tq % ny;
      double v = 0.0;
      for (int s = t; s < nb; ++s) v += T[t * nb + s] * W[s * ny + q];
      W2[t * ny + q] = v;
    }
    __syncthreads();
    for (int iq = tid; iq < rows * ny; iq += NTB) {
      const int i = iq / ny, q = iq % ny;
      double y = Y[(size_t)(j0 + i) * ny + q];
      for (int t = 0; t < nb && t <= i; ++t) {
        const double v = i == t ? 1.0 : V[(size_t)t * m + i];
        y -= v * W2[t * ny + q];
      }
      Y[(size_t)(j0 + i) * ny + q] = y;
    }
    __syncthreads();
  }
}

// 1 / sqrt(x) from the hardware estimate and two Newton steps (double
// precision).
__device__ inline double rsqrt2(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r;
}

// Pair (ci, cj) of round rnd of the circle (round-robin) order on ne
// (even) columns, or false when it touches the padding column ne - 1 >= n.
__device__ inline bool circle_pair(int rnd, int pr, int ne, int n, int& ci, int& cj) {
  if (pr == 0) { ci = rnd; cj = ne - 1; }
  else { ci = (rnd + pr) % (ne - 1); cj = (rnd - pr + ne - 1) % (ne - 1); }
  if (ci > cj) { const int t = ci; ci = cj; cj = t; }
  return cj < n;
}

// Pair schedules of one LDS pass over two column blocks of n1 and n2
// columns (local columns 0..n1-1 and n1..n1+n2-1):
//   SWEEP_ALL    every pair of the n1 + n2 columns (circle order);
//   SWEEP_INTRA  the pairs inside each block, both blocks side by side;
//   SWEEP_CROSS  the n1 n2 pairs between the blocks: in round t column a
//                of the first block meets column (a + t) mod max(n1, n2)
//                of the second.
enum { SWEEP_ALL = 0, SWEEP_INTRA = 1, SWEEP_CROSS = 2 };

// One pass over the columns held in LDS (column stride ld; local column
// j < n1 at slot j, later ones at slot bw + j - n1) in the given schedule:
// one barrier per round.  Returns nonzero (on every thread) when some
// rotation was above the stopping threshold.
__device__ __forceinline__ int lds_sweep(double* Gl, int mg, int n1, int n2, int ld, int bw, int mode, int* flag) {
  const int tid = threadIdx.x;
  const int nl = n1 + n2;
  const int ne = nl + (nl & 1);
  const int e1 = n1 + (n1 & 1), e2 = n2 + (n2 & 1);
  const int mx = n1 > n2 ? n1 : n2;
  const int npairs = mode == SWEEP_ALL ? ne / 2 : (mode == SWEEP_INTRA ? e1 / 2 + e2 / 2 : n1);
  const int rounds = mode == SWEEP_ALL ? ne - 1 : (mode == SWEEP_INTRA ? (e1 > e2 ? e1 : e2) - 1 : mx);
  if (npairs <= 0 || rounds <= 0) return 0;
  const int q = NTB / npairs;
  const int lp = q >= 16 ? 16 : (q >= 8 ? 8 : (q >= 4 ? 4 : (q >= 2 ? 2 : 1)));
  const int gpr = NTB / lp;
  const int grp = tid / lp, li = tid % lp;
  if (tid == 0) *flag = 0;
  __syncthreads();
  for (int rnd = 0; rnd < rounds; ++rnd) {
    for (int pr = grp; pr < npairs; pr += gpr) {
      int ci, cj;
      if (mode == SWEEP_ALL) {
        if (!circle_pair(rnd, pr, ne, nl, ci, cj)) continue;
      } else if (mode == SWEEP_INTRA) {
        if (pr < e1 / 2) {
          if (rnd >= e1 - 1 || !circle_pair(rnd, pr, e1, n1, ci, cj)) continue;
        } else {
          if (rnd >= e2 - 1 || !circle_pair(rnd, pr - e1 / 2, e2, n2, ci, cj)) continue;
          ci += n1;
          cj += n1;
        }
      } else {
        const int b = (pr + rnd) % mx;
        if (b >= n2) continue;
        ci = pr;
        cj = n1 + b;
      }
      double* gi = Gl + (ci < n1 ? ci : bw + ci - n1) * ld;
      double* gj = Gl + (cj < n1 ? cj : bw + cj - n1) * ld;
      // the pair's rows are loaded into registers in one batch (EMAX per
      // lane; longer columns are streamed)
      constexpr int EMAX = 16;
      const bool staged = mg <= lp * EMAX;
      double xr[EMAX], yr[EMAX];
      double al[2] = {0.0, 0.0}, be[2] = {0.0, 0.0}, ga[2] = {0.0, 0.0};
      if (staged) {
#pragma unroll
        for (int u = 0; u < EMAX; ++u) {
          const int i = li + lp * u;
          xr[u] = i < mg ? gi[i] : 0.0;
          yr[u] = i < mg ? gj[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < EMAX; ++u) {
          al[u & 1] += xr[u] * xr[u];
          be[u & 1] += yr[u] * yr[u];
          ga[u & 1] += xr[u] * yr[u];
        }
      } else {
        int t = 0;
        for (int i = li; i < mg; i += lp, ++t) {
          const double x = gi[i], y = gj[i];
          al[t & 1] += x * x;
          be[t & 1] += y * y;
          ga[t & 1] += x * y;
        }
      }
      double sa = al[0] + al[1], sb = be[0] + be[1], sg = ga[0] + ga[1];
      sa = group_sum(sa, lp);
      sb = group_sum(sb, lp);
      sg = group_sum(sg, lp);
      if (sg != 0.0 && sg * sg > (JAC_TOL * JAC_TOL) * (sa * sb)) {
        // Rutishauser's angle from the double angle (d = sb - sa, e = 2 sg):
        // (c, s) parallel to ((1 + |d|/r) / 2, sign(d) e / (2 r)), with 1/r
        // refined to double precision (an inexact angle leaves its error in
        // the pair's orthogonality); the normalisation uses a refined
        // 1/sqrt, so that c^2 + s^2 = 1 to rounding.  Outside the
        // estimate's range of d^2 + e^2 the divisions are exact.
        const double d = sb - sa, e = 2.0 * sg;
        const double r2 = fma(d, d, e * e);
        double h, qv;
        if (r2 < 1.0e300 && r2 > 1.0e-300) {
          const double u = rsqrt2(r2);
          h = fma(0.5 * fabs(d), u, 0.5);
          qv = (d >= 0.0 ? 0.5 : -0.5) * e * u;
        } else {
          const double r = sqrt(r2);
          h = 0.5 + 0.5 * fabs(d) / r;
          qv = (d >= 0.0 ? 0.5 : -0.5) * e / r;
        }
        const double w = rsqrt2(fma(h, h, qv * qv));
        const double c = h * w, s = qv * w;
        if (staged) {
#pragma unroll
          for (int u = 0; u < EMAX; ++u) {
            const int i = li + lp * u;
            if (i < mg) {
              gi[i] = c * xr[u] - s * yr[u];
              gj[i] = s * xr[u] + c * yr[u];
            }
          }
        } else {
          for (int i = li; i < mg; i += lp) {
            const double x = gi[i], y = gj[i];
            gi[i] = c * x - s * y;
            gj[i] = s * x + c * y;
          }
        }
        // a sweep whose rotations all stay below 1e-8 is the last one: the
        // next would be at rounding level (quadratic convergence)
        if (li == 0 && sg * sg > (JAC_CONV_BIG * JAC_CONV_BIG) * (sa * sb)) *flag = 1;
      }
    }
    __syncthreads();
  }
  const int f = *flag;
  __syncthreads();
  return f;
}

// Block one-sided Jacobi on G (mg x ng, column-major, stride cs) in the
// workspace: the columns form blocks of bw.  An outer sweep first rotates
// the pairs inside every block (two blocks per LDS pass), then, for every
// pair of blocks (round-robin over blocks), loads both into LDS (2 bw
// columns), rotates the pairs between them once and writes them back: each
// column pair once per outer sweep, as in the cyclic method.  An outer sweep
// whose rotations all stay below the stopping threshold is the last.  With
// a single block the block is swept in LDS until no pair rotates.
__device__ __forceinline__ void jacobi_blocked(double* G, int mg, int ng, int cs, double* Gl, int* flags) {
  const int tid = threadIdx.x;
  if (ng < 2) return;
  const int ld = mg | 1;
  int bw = PANEL_DOUBLES / (2 * ld);
  if (bw > 32) bw = 32;
  if (bw < 1) bw = 1;
  const int nblk = (ng + bw - 1) / bw;
  auto load = [&](int b, int slot) {
    const int c0 = b * bw, nc = ng - c0 < bw ? ng - c0 : bw;
    for (int idx = tid; idx < nc * mg; idx += NTB) {
      const int j = idx / mg, i = idx % mg;
      Gl[(slot * bw + j) * ld + i] = G[(size_t)(c0 + j) * cs + i];
    }
    return nc;
  };
  auto store = [&](int b, int slot, int nc) {
    const int c0 = b * bw;
    for (int idx = tid; idx < nc * mg; idx += NTB) {
      const int j = idx / mg, i = idx % mg;
      G[(size_t)(c0 + j) * cs + i] = Gl[(slot * bw + j) * ld + i];
    }
  };
  if (nblk == 1) {
    load(0, 0);
    __syncthreads();
    for (int sweep = 0; sweep < JAC_MAX_SWEEPS; ++sweep)
      if (!lds_sweep(Gl, mg, ng, 0, ld, bw, SWEEP_ALL, flags)) break;
    store(0, 0, ng);
    __syncthreads();
    return;
  }
  const int nbe = nblk + (nblk & 1);
  for (int sweep = 0; sweep < JAC_MAX_SWEEPS; ++sweep) {
    int any = 0;
    for (int b = 0; b < nblk; b += 2) {
      const int n1 = load(b, 0), n2 = b + 1 < nblk ? load(b + 1, 1) : 0;
      __syncthreads();
      any |= lds_sweep(Gl, mg, n1, n2, ld, bw, SWEEP_INTRA, flags + 1);
      store(b, 0, n1);
      if (n2) store(b + 1, 1, n2);
      __syncthreads();
    }
    for (int rnd = 0; rnd < nbe - 1; ++rnd)
      for (int pr = 0; pr < nbe / 2; ++pr) {
        int b1, b2;
        if (pr == 0) { b1 = rnd; b2 = nbe - 1; }
        else { b1 = (rnd + pr) % (nbe - 1); b2 = (rnd - pr + nbe - 1) % (nbe - 1); }
        if (b1 >= nblk || b2 >= nblk) continue;
        const int n1 = load(b1, 0), n2 = load(b2, 1);
        __syncthreads();
        any |= lds_sweep(Gl, mg, n1, n2, ld, bw, SWEEP_CROSS, flags + 1);
        store(b1, 0, n1);
        store(b2, 1, n2);
        __syncthreads();
      }
    if (!any) break;
  }
}

}  // namespace

__global__ void __launch_bounds__(NTB) k_compress_big(Prob P, int dir, int r, const double* __restrict__ theta,
                                                     const uint8_t* __restrict__ configs, double* ws,
                                                     int32_t* status) {
  __shared__ Geo geo;
  __shared__ double red[NTB];
  __shared__ double panel[PANEL_DOUBLES];
  __shared__ double Tm[NBMAX * NBMAX];
  __shared__ double sig[CD_MAX];
  __shared__ int rnk[CD_MAX];
  __shared__ int flags[2];
  __shared__ int sa[MAX_L], sp[MAX_L], sb[MAX_L];
  __shared__ int rst_n[MAX_L];   // columns of site c's QR matrix (R_c is sb[c] x rst_n[c])
  const int tid = threadIdx.x;
  const int ch = blockIdx.x;
  if (tid == 0) build_geo(P, geo);
  __syncthreads();
  ChainWS w = chain_ws(P, ws, ch);
  double* base = ws + (size_t)ch * P.chain_stride;
  double* taus_all = base + P.off_tau;
  double* T_all = base + P.off_T;
  const int cd = P.chi * P.D;
  const uint8_t* cfg = configs + (size_t)ch * P.N;
  double* bnd = dir == 0 ? w.top : w.bot;
  double* lsb = dir == 0 ? w.lstop : w.lsbot;
  double* outT = bnd + (size_t)r * P.L2 * P.TS;
  const bool has_prev = dir == 0 ? (r > 0) : (r < P.L1 - 1);
  const int rp = dir == 0 ? r - 1 : r + 1;
  const double ls_prev = has_prev ? lsb[rp] : 0.0;

  // 1. site 0 absorbed straight into its QR matrix (rows (x, p), column-major)
  {
    int a0, p0, b0;
    int Dl, Du, Dr, Dd;
    leg_dims(P, r, 0, Dl, Du, Dr, Dd);
    const int pp = dir == 0 ? Dd : Du;
    const int a = (has_prev ? geo.ba[dir][rp][0] : 1) * Dl;
    const int m0 = a * pp;
    absorb_site_to(P, geo, dir, r, 0, theta, cfg, bnd, has_prev, rp, w.B, pp, 1, m0, a0, p0, b0);
    if (tid == 0) { sa[0] = a0; sp[0] = p0; sb[0] = b0; }
  }
  __syncthreads();

  // 2. left-to-right QR in the one QR matrix X (w.B); X_{c+1} = R_c B_{c+1}
  // by MFMA tiles.  R_c is kept for every site: the truncation sweep rebuilds
  // X_{c} from it to apply Q_c again, instead of keeping every site's
  // reflectors (which would take L2 QR matrices per chain).
  // QR matrix of site c: its own slot when every site's reflectors are kept,
  // else the one slot (rebuilt when needed)
  auto xslot = [&](int c) { return P.refl_store ? w.B + (size_t)c * P.BS : w.B; };
  double* Rst = base + P.off_Rst;
  // B_c absorbed into dst, row-major [y][p][col]; returns its dims
  auto absorb_rm = [&](int c, double* dst, int& a1, int& p1, int& b1) {
    int Dl, Du, Dr, Dd;
    leg_dims(P, r, c, Dl, Du, Dr, Dd);
    const int pp = dir == 0 ? Dd : Du;
    const int bb = (has_prev ? geo.bb[dir][rp][c] : 1) * Dr;
    absorb_site_to(P, geo, dir, r, c, theta, cfg, bnd, has_prev, rp, dst, (int64_t)pp * bb, bb, 1, a1, p1, b1);
  };
  // X = R B (k x n times the absorbed site [n][p1][b1]) into the column-major
  // QR layout: X[col * m' + x * p1 + q] = sum_y R[x][y] B[y][q][col], m' = k p1
  auto rb_product = [&](double* X, const double* Rr, int k, int n, const double* Bsrc, int p1, int b1) {
    wg_gemm<double>(X, mstride(p1), Map2{b1, 1, k * p1}, Rr, mstride(n), mid(), Bsrc, mstride(p1 * b1), mid(), k,
                    p1 * b1, n);
  };
  for (int c = 0; c < P.L2 - 1; ++c) {
    const int m = sa[c] * sp[c], n = sb[c];
    const int k = m < n ? m : n;
    double* X = xslot(c);
    qr_blocked(X, m, n, taus_all + (size_t)c * cd, T_all + (size_t)c * cd * NBMAX, panel, Tm, red);
    // R_c (k x n, row-major, zero below the diagonal); kept per site only
    // when the reflectors are rebuilt
    double* Rr = P.refl_store ? w.R : Rst + (size_t)c * cd * cd;
    for (int idx = tid; idx < k * n; idx += NTB) {
      const int i = idx / n, j = idx % n;
      Rr[idx] = j >= i ? X[(size_t)j * m + i] : 0.0;
    }
    int a1, p1, b1;
    absorb_rm(c + 1, w.tmp, a1, p1, b1);
    __syncthreads();
    if (a1 != n) set_status(status, PEPS_ERR_UNSUPPORTED);   // bond of the absorbed row: cannot differ
    rb_product(xslot(c + 1), Rr, k, n, w.tmp, p1, b1);
    if (tid == 0) {
      rst_n[c] = n;
      sb[c] = k;
      sa[c + 1] = k;
      sp[c + 1] = p1;
      sb[c + 1] = b1;
    }
    __syncthreads();
  }
  // the last site as the first truncation matrix: row-major a x (p b)
  {
    const int c = P.L2 - 1;
    const int a = sa[c], pp = sp[c], b = sb[c], m = a * pp;
    const double* X = xslot(c);
    for (int idx = tid; idx < a * pp * b; idx += NTB) {
      const int i = idx / (pp * b), e = idx % (pp * b), p = e / b, col = e % b;
      w.tmp[idx] = X[(size_t)col * m + i * pp + p];
    }
    __syncthreads();
  }

  // 3. right-to-left truncation to chi
  for (int c = P.L2 - 1; c >= 1; --c) {
    const int a = sa[c], nb = sp[c] * sb[c];
    // G = M^T when M has no more rows than columns: its columns become V S
    // and U S = M V_k follows without accumulating rotations; else G = M
    // with the rotations accumulated into V (ng = nb is then small)
    const bool tr = a <= nb;
    const int mg = tr ? nb : a, ng = tr ? a : nb;
    const int cs = mg | 1;
    double* G = w.X;
    double* V = w.X + (size_t)cs * ng;
    const double* M = w.tmp;
    for (int idx = tid; idx < mg * ng; idx += NTB) {
      const int j = idx / mg, i = idx % mg;
      G[(size_t)j * cs + i] = tr ? M[(size_t)j * nb + i] : M[(size_t)i * nb + j];
    }
    if (!tr)
      for (int idx = tid; idx < ng * ng; idx += NTB) {
        const int j = idx / ng, i = idx % ng;
        V[idx] = (i == j) ? 1.0 : 0.0;
      }
    __syncthreads();
    if (tr) jacobi_blocked(G, mg, ng, cs, panel, flags);
    else wg_jacobi(G, mg, ng, cs, V, ng, flags);
    for (int j = tid; j < ng; j += NTB) {
      double s = 0.0;
      for (int i = 0; i < mg; ++i) s += G[(size_t)j * cs + i] * G[(size_t)j * cs + i];
      sig[j] = rank_norm(s, status);
    }
    __syncthreads();
    for (int j = tid; j < ng; j += NTB) {
      int rk = 0;
      for (int q = 0; q < ng; ++q)
        if (sig[q] > sig[j] || (sig[q] == sig[j] && q < j)) ++rk;
      rnk[j] = rk;
    }
    __syncthreads();
    const int k2 = P.chi < ng ? P.chi : ng;
    double* Vt = outT + (size_t)c * P.TS;
    double* US = w.R;   // a x k2, row-major
    if (tr) {
      for (int idx = tid; idx < nb * ng; idx += NTB) {
        const int e = idx / ng, j = idx % ng;
        const int q = rnk[j];
        if (q < k2) Vt[q * nb + e] = sig[j] > 0.0 ? G[(size_t)j * cs + e] / sig[j] : 0.0;
      }
      __syncthreads();
      for (int idx = tid; idx < a * k2; idx += NTB) {
        const int i = idx / k2, q = idx % k2;
        double s = 0.0;
        for (int e = 0; e < nb; ++e) s += M[(size_t)i * nb + e] * Vt[q * nb + e];
        US[idx] = s;
      }
    } else {
      for (int idx = tid; idx < a * ng; idx += NTB) {
        const int i = idx / ng, j = idx % ng;
        const int q = rnk[j];
        if (q < k2) US[i * k2 + q] = G[(size_t)j * cs + i];
      }
      for (int idx = tid; idx < nb * ng; idx += NTB) {
        const int e = idx / ng, j = idx % ng;
        const int q = rnk[j];
        if (q < k2) Vt[q * nb + e] = V[(size_t)j * ng + e];
      }
    }
    __syncthreads();
    // A_{c-1} <- Q_{c-1} [U S; 0]: m2 x k2 row-major into tmp
    const int m2 = sa[c - 1] * sp[c - 1];
    const int kq = sb[c - 1];
    for (int idx = tid; idx < m2 * k2; idx += NTB) {
      const int i = idx / k2, q = idx % k2;
      w.tmp[idx] = i < a ? US[i * k2 + q] : 0.0;
    }
    // X_{c-1} rebuilt exactly as in the first sweep (the same absorption,
    // product and QR, so the same reflectors), then Q_{c-1} applied
    double* X = xslot(c - 1);
    if (P.refl_store) {
      // kept from the first sweep
    } else if (c - 1 == 0) {
      int a0, p0, b0;
      absorb_site_to(P, geo, dir, r, 0, theta, cfg, bnd, has_prev, rp, X, sp[0], 1, (int64_t)sa[0] * sp[0], a0, p0,
                     b0);
    } else {
      // X_{c-1} = R_{c-2} B_{c-1}: R_{c-2} is sa[c-1] x rst_n[c-2]
      int a1, p1, b1;
      absorb_rm(c - 1, w.X, a1, p1, b1);
      __syncthreads();
      rb_product(X, Rst + (size_t)(c - 2) * cd * cd, sa[c - 1], rst_n[c - 2], w.X, p1, b1);
    }
    __syncthreads();
    if (!P.refl_store)
      qr_blocked(X, m2, rst_n[c - 1], taus_all + (size_t)(c - 1) * cd, T_all + (size_t)(c - 1) * cd * NBMAX, panel,
                 Tm, red);
    apply_q_blocked(X, m2, kq, T_all + (size_t)(c - 1) * cd * NBMAX, w.tmp, k2, panel);
    if (tid == 0) {
      sb[c - 1] = k2;
      sa[c] = k2;
    }
    __syncthreads();
  }

  // 4. normalise site 0 and accumulate the log-scale
  const int tot0 = sa[0] * sp[0] * sb[0];
  double part = 0.0;
  for (int idx = tid; idx < tot0; idx += NTB) part += w.tmp[idx] * w.tmp[idx];
  const double nrm = sqrt(block_sum_b(part, red));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int idx = tid; idx < tot0; idx += NTB) outT[idx] = w.tmp[idx] * inv;
  if (tid == 0) {
    lsb[r] = nrm > 0.0 ? ls_prev + log(nrm) : -INFINITY;
    for (int c = 0; c < P.L2; ++c)
      if (sa[c] != geo.ba[dir][r][c] || sb[c] != geo.bb[dir][r][c]) set_status(status, PEPS_ERR_UNSUPPORTED);
  }
  if (P.mixed) {
    __syncthreads();
    float* o32 = (float*)(ws + (size_t)ch * P.chain_stride + (dir == 0 ? P.off_top32 : P.off_bot32)) +
                 (size_t)r * P.L2 * P.TS;
    for (int idx = tid; idx < P.L2 * P.TS; idx += NTB) o32[idx] = (float)outT[idx];
  }
}

size_t compress_big_T_doubles(const Prob& P) { return (size_t)P.L2 * P.chi * P.D * NBMAX; }

hipError_t launch_compress_big(const Prob& P, int n, int dir, int r, const double* theta, const uint8_t* configs,
                               double* ws, int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_compress_big, dim3(n), dim3(NTB), 0, st, P, dir, r, theta, configs, ws, status);
  return hipGetLastError();
}

}  // namespace peps
