// Workgroup-level dense factorisations in FP64, on matrices in LDS or in a
// workspace in device memory.
//
//  * Householder QR (Golub & Van Loan, Alg. 5.2.1, LAPACK dgeqr2/dorg2r
//    conventions): reflector H = I - tau v v^T with v_0 = 1, R's diagonal
//    beta = -sign(alpha) ||x||, explicit thin Q formed in place by backward
//    accumulation.  Handles rank-deficient and zero columns (tau = 0).
//  * One-sided Jacobi SVD (Hestenes 1958; Rutishauser rotation; Demmel &
//    Veselic 1992 for its accuracy): pairs of columns are rotated until
//    every pair is orthogonal to a relative tolerance, the rotations being
//    accumulated into an orthogonal matrix.  Pairs are scheduled by the
//    round-robin (circle) ordering so that all pairs of one round are
//    disjoint and run in parallel, eight lanes per pair.
#pragma once

#include "peps_common.hpp"

namespace peps {

// ---------------------------------------------------------------------------
// QR of X (m x n, row-major, leading dimension ld) in LDS.  On return the
// upper triangle of the first k = min(m, n) rows holds R, the strict lower
// part the reflectors, tau[0..k) their scalars.  red: NT doubles of LDS.
__device__ inline void wg_householder(double* X, int m, int n, int ld, double* tau, double* red) {
  const int tid = threadIdx.x;
  const int k = m < n ? m : n;
  for (int j = 0; j < k; ++j) {
    // sigma2 = sum_{i>j} X[i][j]^2
    double part = 0.0;
    for (int i = j + 1 + tid; i < m; i += NT) {
      double x = X[i * ld + j];
      part += x * x;
    }
    double sigma2 = wg_sum(part, red);
    double alpha = X[j * ld + j];
    double t = 0.0, scale = 0.0, beta = alpha;
    if (sigma2 > 0.0) {
      double nrm = sqrt(alpha * alpha + sigma2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // every thread holds the same t / scale / beta (same inputs, same ops)
    if (t != 0.0) {
      for (int i = j + 1 + tid; i < m; i += NT) X[i * ld + j] *= scale;
    }
    __syncthreads();
    if (tid == 0) {
      X[j * ld + j] = beta;
      tau[j] = t;
    }
    if (t != 0.0) {
      // w_col = X[j][col] + sum_{i>j} v_i X[i][col]; X[i][col] -= t v_i w_col
      const int ncol = n - j - 1;
      if (ncol > 0) {
        // threads are split into column lanes x row groups
        const int groups = NT / 64 >= 1 ? NT / 64 : 1;  // 4 row groups of 64 columns
        for (int cbase = 0; cbase < ncol; cbase += 64) {
          int cc = tid % 64, g = tid / 64;
          int col = j + 1 + cbase + cc;
          double w = 0.0;
          if (cbase + cc < ncol) {
            if (g == 0) w = X[j * ld + col];
            for (int i = j + 1 + g; i < m; i += groups) w += X[i * ld + j] * X[i * ld + col];
          }
          red[tid] = w;
          __syncthreads();
          if (g == 0 && cbase + cc < ncol) {
            double s = red[cc];
            for (int q = 1; q < groups; ++q) s += red[q * 64 + cc];
            red[NT - 64 + cc] = s;  // stash (row group 3 slots already consumed)
          }
          __syncthreads();
          if (cbase + cc < ncol) {
            double wt = t * red[NT - 64 + cc];
            if (g == 0) X[j * ld + col] -= wt;
            for (int i = j + 1 + g; i < m; i += groups) X[i * ld + col] -= X[i * ld + j] * wt;
          }
          __syncthreads();
        }
      }
    }
    __syncthreads();
  }
}

// Overwrite the reflectors of wg_householder with the explicit thin Q
// (m x k), in place (columns 0..k-1; row-major, leading dimension ld).
__device__ inline void wg_form_q(double* X, int m, int n, int ld, const double* tau, double* red) {
  const int tid = threadIdx.x;
  const int k = m < n ? m : n;
  for (int j = k - 1; j >= 0; --j) {
    const double t = tau[j];
    const int ncol = k - j - 1;
    // apply H_j to columns j+1..k-1 (rows j..m-1), v = (1, X[j+1..m-1][j])
    if (ncol > 0 && t != 0.0) {
      const int groups = NT / 64;
      for (int cbase = 0; cbase < ncol; cbase += 64) {
        int cc = tid % 64, g = tid / 64;
        int col = j + 1 + cbase + cc;
        double w = 0.0;
        if (cbase + cc < ncol) {
          if (g == 0) w = X[j * ld + col];
          for (int i = j + 1 + g; i < m; i += groups) w += X[i * ld + j] * X[i * ld + col];
        }
        red[tid] = w;
        __syncthreads();
        if (g == 0 && cbase + cc < ncol) {
          double s = red[cc];
          for (int q = 1; q < groups; ++q) s += red[q * 64 + cc];
          red[NT - 64 + cc] = s;
        }
        __syncthreads();
        if (cbase + cc < ncol) {
          double wt = t * red[NT - 64 + cc];
          if (g == 0) X[j * ld + col] -= wt;
          for (int i = j + 1 + g; i < m; i += groups) X[i * ld + col] -= X[i * ld + j] * wt;
        }
        __syncthreads();
      }
    }
    // column j itself: e_j - t v
    for (int i = tid; i < m; i += NT) {
      double v;
      if (i < j) v = 0.0;
      else if (i == j) v = 1.0 - t;
      else v = -t * X[i * ld + j];
      X[i * ld + j] = v;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// One-sided Jacobi on G (mg x ng, column-major with column stride cs) with
// accumulation into V (ng x ng, column-major, stride vs), V = I on entry.
// On return the columns of G are mutually orthogonal (to tolerance) and
// G_in V = G_out.
constexpr int JAC_LANES = 8;
constexpr int JAC_MAX_SWEEPS = 40;
constexpr double JAC_TOL = 2.0e-15;

__device__ inline void wg_jacobi(double* G, int mg, int ng, int cs, double* V, int vs, int* flags) {
  const int tid = threadIdx.x;
  if (ng < 2) return;
  const int ne = ng + (ng & 1);
  const int npairs = ne / 2;
  const int gpr = (int)blockDim.x / JAC_LANES;  // groups per pass
  const int grp = tid / JAC_LANES, lane = tid % JAC_LANES;
  if (tid == 0) { flags[0] = 0; flags[1] = 0; }
  __syncthreads();
  for (int sweep = 0; sweep < JAC_MAX_SWEEPS; ++sweep) {
    const int fl = sweep & 1;
    for (int rnd = 0; rnd < ne - 1; ++rnd) {
      for (int pbase = 0; pbase < npairs; pbase += gpr) {
        const int p = pbase + grp;
        int ci = -1, cj = -1;
        if (p < npairs) {
          if (p == 0) { ci = rnd; cj = ne - 1; }
          else { ci = (rnd + p) % (ne - 1); cj = (rnd - p + ne - 1) % (ne - 1); }
          if (ci >= ng || cj >= ng) { ci = -1; }
          if (ci > cj && ci >= 0) { int t = ci; ci = cj; cj = t; }
        }
        double al = 0.0, be = 0.0, ga = 0.0;
        if (ci >= 0) {
          const double* gi = G + (size_t)ci * cs;
          const double* gj = G + (size_t)cj * cs;
          for (int i = lane; i < mg; i += JAC_LANES) {
            double x = gi[i], y = gj[i];
            al += x * x; be += y * y; ga += x * y;
          }
        }
        // butterfly within the 8 lanes of the group: identical bits on all
        for (int off = 1; off < JAC_LANES; off <<= 1) {
          al += __shfl_xor(al, off, JAC_LANES);
          be += __shfl_xor(be, off, JAC_LANES);
          ga += __shfl_xor(ga, off, JAC_LANES);
        }
        if (ci >= 0 && ga != 0.0 && fabs(ga) > JAC_TOL * sqrt(al) * sqrt(be)) {
          double zeta = (be - al) / (2.0 * ga);
          double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
          double c = 1.0 / sqrt(1.0 + t * t);
          double s = c * t;
          double* gi = G + (size_t)ci * cs;
          double* gj = G + (size_t)cj * cs;
          for (int i = lane; i < mg; i += JAC_LANES) {
            double x = gi[i], y = gj[i];
            gi[i] = c * x - s * y;
            gj[i] = s * x + c * y;
          }
          double* vi = V + (size_t)ci * vs;
          double* vj = V + (size_t)cj * vs;
          for (int i = lane; i < ng; i += JAC_LANES) {
            double x = vi[i], y = vj[i];
            vi[i] = c * x - s * y;
            vj[i] = s * x + c * y;
          }
          if (lane == 0) flags[fl] = 1;
        }
        __syncthreads();
      }
    }
    __syncthreads();
    const bool done = flags[fl] == 0;
    __syncthreads();
    if (tid == 0) flags[fl] = 0;
    __syncthreads();
    if (done) break;
  }
}

}  // namespace peps
