// Simple-update imaginary-time evolution (the high-temperature alternative
// to SR, after Appendix A; the scheme of Jiang, Weng and Xiang): one
// first-order Trotter step of tau applies exp(-tau calH_b) to every
// nearest-neighbour bond, in four groups of disjoint bonds (horizontal with
// c even, c odd; vertical with r even, r odd), with bond weights lambda
// standing in for the environment.
//
// One workgroup per bond of a group.  For the bond (i, j) with leg li of i
// and lj of j:
//   1. X_i = T_i as (other legs) x (S_i, b) with the other legs multiplied by
//      their weights, and X_j likewise;
//   2. X = Q R from one-sided Jacobi: X V = G, sigma_c = |G_c|,
//      Q = G / sigma, R = diag(sigma) V^T (no QR kernel needed);
//   3. Theta[(c_i, S_i'), (S_j', c_j)] = sum G2 R_i lambda_b R_j with the
//      doubled gate G2 = exp(-tau J h) (x) exp(-tau J h), h = S_i.S_j, from
//      its closed form: e^{-tau J/4} on the triplet, e^{3 tau J/4} on the
//      singlet;
//   4. one-sided Jacobi on Theta with V accumulated, the D largest singular
//      values kept (NaN-safe ranking), lambda_b = kept / largest;
//   5. T_i = Q_i U, T_j = Q_j V, the other legs divided by their weights
//      again (a weight at or below 1e-12 of its bond's largest counts as 0).
// Work matrices live in the workspace (one slice per workgroup); for D <= 4
// the Jacobi rotations run on copies in LDS.
#include <math.h>

#include "peps_common.hpp"
#include "peps_kernels.hpp"
#include "peps_linalg.hpp"

namespace peps {

namespace {

constexpr int SU_NT = 256;
constexpr double SU_LAMBDA_CUT = 1.0e-12;
constexpr int SU_LDS_NT = 64;    // two-site matrices up to 64 x 64 (D <= 4) are rotated in LDS

struct SuBond {
  int i, j, li, lj, k;   // sites, legs (0 l, 1 u, 2 r, 3 d) and bond index
};

// Bond `e` of group g (0: horizontal, c even; 1: horizontal, c odd;
// 2: vertical, r even; 3: vertical, r odd), bonds of a group row-major.
__host__ __device__ inline int su_group_size(const Prob& P, int g) {
  switch (g) {
    case 0: return P.L1 * (P.L2 / 2);
    case 1: return P.L1 * ((P.L2 - 1) / 2);
    case 2: return (P.L1 / 2) * P.L2;
    default: return ((P.L1 - 1) / 2) * P.L2;
  }
}

__device__ inline SuBond su_bond(const Prob& P, int g, int e) {
  SuBond b;
  if (g < 2) {
    const int per = g == 0 ? P.L2 / 2 : (P.L2 - 1) / 2;
    const int r = e / per, c = 2 * (e % per) + g;
    b.i = r * P.L2 + c;
    b.j = b.i + 1;
    b.li = 2;
    b.lj = 0;
    b.k = r * (P.L2 - 1) + c;
  } else {
    const int r = 2 * (e / P.L2) + (g - 2), c = e % P.L2;
    b.i = r * P.L2 + c;
    b.j = b.i + P.L2;
    b.li = 3;
    b.lj = 1;
    b.k = P.L1 * (P.L2 - 1) + r * P.L2 + c;
  }
  return b;
}

// Bond index on leg `leg` of site (r, c), or -1 on an open boundary.
__device__ inline int leg_bond(const Prob& P, int r, int c, int leg) {
  switch (leg) {
    case 0: return c > 0 ? r * (P.L2 - 1) + c - 1 : -1;
    case 1: return r > 0 ? P.L1 * (P.L2 - 1) + (r - 1) * P.L2 + c : -1;
    case 2: return c < P.L2 - 1 ? r * (P.L2 - 1) + c : -1;
    default: return r < P.L1 - 1 ? P.L1 * (P.L2 - 1) + r * P.L2 + c : -1;
  }
}

__device__ inline int param_offset(const Prob& P, int site) {
  int po = 0;
  for (int s = 0; s < site; ++s) po += P.d2 * block_size(P, s / P.L2, s % P.L2);
  return po;
}

// Weight of index x on leg `leg` of site (r, c) (1 on a boundary or on the
// bond being updated); inverse = 1 gives the cut inverse.
__device__ inline double leg_weight(const Prob& P, const double* lam, int r, int c, int leg, int skip, int x,
                                    bool inverse) {
  if (leg == skip) return 1.0;
  const int k = leg_bond(P, r, c, leg);
  if (k < 0) return 1.0;
  const double v = lam[(size_t)k * P.D + x];
  if (!inverse) return v;
  double mx = 0.0;
  for (int t = 0; t < P.D; ++t) mx = fmax(mx, lam[(size_t)k * P.D + t]);
  return v > SU_LAMBDA_CUT * mx ? 1.0 / v : 0.0;
}

// exp(-tau J S_i.S_j) on (s_i, s_j), index s_i * 2 + s_j (digit 0 = up).
__device__ inline double gate1(double et, double es, int a, int b) {
  const int si = a >> 1, sj = a & 1, ti = b >> 1, tj = b & 1;
  double ss = 0.0;   // <si sj| S_i.S_j |ti tj>
  if (si == ti && sj == tj) ss = (si == sj) ? 0.25 : -0.25;
  else if (si != sj && ti == sj && tj == si) ss = 0.5;
  const double id = (a == b) ? 1.0 : 0.0;
  // e^{-tau J/4} (3/4 + S.S) + e^{3 tau J/4} (1/4 - S.S)
  return et * (0.75 * id + ss) + es * (0.25 * id - ss);
}

// Doubled gate entry <(Si', Sj')| G2 |(Si, Sj)>, S = s * 2 + s'.
__device__ inline double gate2(double et, double es, int Sip, int Sjp, int Si, int Sj) {
  const int ket_p = ((Sip >> 1) << 1) | (Sjp >> 1), ket = ((Si >> 1) << 1) | (Sj >> 1);
  const int bra_p = ((Sip & 1) << 1) | (Sjp & 1), bra = ((Si & 1) << 1) | (Sj & 1);
  return gate1(et, es, ket_p, ket) * gate1(et, es, bra_p, bra);
}

struct SuSite {
  int r, c, li, dims[4], m, po;   // m: product of the three other leg dimensions
};

__device__ inline SuSite su_site(const Prob& P, int i, int li) {
  SuSite s;
  s.r = i / P.L2;
  s.c = i % P.L2;
  s.li = li;
  leg_dims(P, s.r, s.c, s.dims[0], s.dims[1], s.dims[2], s.dims[3]);
  s.m = 1;
  for (int l = 0; l < 4; ++l)
    if (l != li) s.m *= s.dims[l];
  s.po = param_offset(P, i);
  return s;
}

// Element (S, x0, x1, x2, x3) of T in [S][l][u][r][d] order.
__device__ inline size_t t_index(const SuSite& s, int S, const int* x) {
  return ((((size_t)S * s.dims[0] + x[0]) * s.dims[1] + x[1]) * s.dims[2] + x[2]) * s.dims[3] + x[3];
}

// Leg indices of row o of the (other legs) matrix and bond index b.
__device__ inline void su_legs(const SuSite& s, int o, int b, int* x) {
  for (int l = 3; l >= 0; --l) {
    if (l == s.li) { x[l] = b; continue; }
    x[l] = o % s.dims[l];
    o /= s.dims[l];
  }
}

// X (m x n, column-major, n = 4 D, column S * D + b) from T with the other
// legs weighted.
__device__ void su_gather(const Prob& P, const SuSite& s, const double* theta, const double* lam, double* X) {
  const int n = P.d2 * P.D;
  for (int idx = threadIdx.x; idx < s.m * n; idx += blockDim.x) {
    const int col = idx / s.m, o = idx % s.m;
    const int S = col / P.D, b = col % P.D;
    int x[4];
    su_legs(s, o, b, x);
    double w = 1.0;
    for (int l = 0; l < 4; ++l) w *= leg_weight(P, lam, s.r, s.c, l, s.li, x[l], false);
    X[(size_t)col * s.m + o] = theta[s.po + t_index(s, S, x)] * w;
  }
}

// G = X V (in place), V = I on entry: then sigma, Q = G / sigma (in place),
// and R (n x n, row-major) = diag(sigma) V^T.
// With `lds` (room for m n + n n doubles) the rotations run on copies there.
__device__ void su_factor(const Prob& P, const SuSite& s, double* X, double* V, double* R, double* sig,
                          int* flags, int32_t* status, double* lds) {
  const int n = P.d2 * P.D;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) V[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
  __syncthreads();
  if (lds) {
    double* Xl = lds;
    double* Vl = lds + (size_t)s.m * n;
    for (int idx = threadIdx.x; idx < s.m * n; idx += blockDim.x) Xl[idx] = X[idx];
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) Vl[idx] = V[idx];
    __syncthreads();
    wg_jacobi(Xl, s.m, n, s.m, Vl, n, flags);
    for (int idx = threadIdx.x; idx < s.m * n; idx += blockDim.x) X[idx] = Xl[idx];
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) V[idx] = Vl[idx];
    __syncthreads();
  } else {
    wg_jacobi(X, s.m, n, s.m, V, n, flags);
  }
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double q = 0.0;
    for (int o = 0; o < s.m; ++o) q += X[(size_t)c * s.m + o] * X[(size_t)c * s.m + o];
    if (!isfinite(q)) set_status(status, PEPS_ERR_NONFINITE);
    sig[c] = sqrt(q);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < s.m * n; idx += blockDim.x) {
    const int c = idx / s.m;
    X[idx] = sig[c] > 0.0 ? X[idx] / sig[c] : 0.0;
  }
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int c = idx / n, col = idx % n;   // R[c][col] = sigma_c V[col][c]
    R[idx] = sig[c] * V[(size_t)c * n + col];
  }
  __syncthreads();
}

// T (site layout) = sum_c Q[o][c] W[c][(S, k)] with the other legs divided
// by their weights; W(c, S, k) given by a functor.
template <typename F>
__device__ void su_scatter(const Prob& P, const SuSite& s, const double* Q, const double* lam, double* theta, F W) {
  const int n = P.d2 * P.D;
  for (int idx = threadIdx.x; idx < s.m * n; idx += blockDim.x) {
    const int col = idx / s.m, o = idx % s.m;
    const int S = col / P.D, kk = col % P.D;
    double v = 0.0;
    for (int c = 0; c < n; ++c) v += Q[(size_t)c * s.m + o] * W(c, S, kk);
    int x[4];
    su_legs(s, o, kk, x);
    double w = 1.0;
    for (int l = 0; l < 4; ++l) w *= leg_weight(P, lam, s.r, s.c, l, s.li, x[l], true);
    theta[s.po + t_index(s, S, x)] = v * w;
  }
}

}  // namespace

__global__ void __launch_bounds__(SU_NT) k_su_bond(Prob P, int group, double* theta, double* lam, double et,
                                                 double es, double* ws, size_t ws_stride, int32_t* status) {
  __shared__ SuSite si, sj;
  __shared__ SuBond bd;
  __shared__ int flags[2];
  __shared__ double sig_i[4 * MAX_SU_D], sig_j[4 * MAX_SU_D], sig_t[16 * MAX_SU_D];
  __shared__ int keep[MAX_SU_D];
  const int n = P.d2 * P.D, nt = 4 * n;
  if (threadIdx.x == 0) {
    bd = su_bond(P, group, blockIdx.x);
    si = su_site(P, bd.i, bd.li);
    sj = su_site(P, bd.j, bd.lj);
  }
  __syncthreads();
  double* Xi = ws + blockIdx.x * ws_stride;
  double* Xj = Xi + (size_t)si.m * n;
  double* Vi = Xj + (size_t)sj.m * n;
  double* Vj = Vi + (size_t)n * n;
  double* Ri = Vj + (size_t)n * n;
  double* Rj = Ri + (size_t)n * n;
  double* Th = Rj + (size_t)n * n;
  double* Vt = Th + (size_t)nt * nt;
  su_gather(P, si, theta, lam, Xi);
  su_gather(P, sj, theta, lam, Xj);
  __syncthreads();
  extern __shared__ double su_lds[];
  const bool small = nt <= SU_LDS_NT;   // dynamic LDS of 2 nt^2 doubles, >= m n + n n for D <= 4
  su_factor(P, si, Xi, Vi, Ri, sig_i, flags, status, small ? su_lds : nullptr);
  su_factor(P, sj, Xj, Vj, Rj, sig_j, flags, status, small ? su_lds : nullptr);
  // Theta (nt x nt, column-major): row (c_i, S_i'), column (S_j', c_j)
  const double* lb = lam + (size_t)bd.k * P.D;
  for (int idx = threadIdx.x; idx < nt * nt; idx += blockDim.x) {
    const int q = idx / nt, rrow = idx % nt;
    const int ci = rrow / 4, Sip = rrow % 4, Sjp = q / n, cj = q % n;
    double v = 0.0;
    for (int Si = 0; Si < 4; ++Si)
      for (int Sj = 0; Sj < 4; ++Sj) {
        const double g = gate2(et, es, Sip, Sjp, Si, Sj);
        if (g == 0.0) continue;
        double acc = 0.0;
        for (int b = 0; b < P.D; ++b) acc += Ri[(size_t)ci * n + Si * P.D + b] * lb[b] * Rj[(size_t)cj * n + Sj * P.D + b];
        v += g * acc;
      }
    Th[(size_t)q * nt + rrow] = v;
  }
  for (int idx = threadIdx.x; idx < nt * nt; idx += blockDim.x) Vt[idx] = (idx / nt == idx % nt) ? 1.0 : 0.0;
  __syncthreads();
  if (small) {
    // small two-site matrices: the rotations run on copies in LDS
    double* Tl = su_lds;
    double* Vl = su_lds + nt * nt;
    for (int idx = threadIdx.x; idx < nt * nt; idx += blockDim.x) {
      Tl[idx] = Th[idx];
      Vl[idx] = Vt[idx];
    }
    __syncthreads();
    wg_jacobi(Tl, nt, nt, nt, Vl, nt, flags);
    for (int idx = threadIdx.x; idx < nt * nt; idx += blockDim.x) {
      Th[idx] = Tl[idx];
      Vt[idx] = Vl[idx];
    }
    __syncthreads();
  } else {
    wg_jacobi(Th, nt, nt, nt, Vt, nt, flags);
  }
  for (int q = threadIdx.x; q < nt; q += blockDim.x) {
    double ssq = 0.0;
    for (int r = 0; r < nt; ++r) ssq += Th[(size_t)q * nt + r] * Th[(size_t)q * nt + r];
    sig_t[q] = rank_norm(ssq, status);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nt; q += blockDim.x) {
    int rk = 0;
    for (int t = 0; t < nt; ++t)
      if (sig_t[t] > sig_t[q] || (sig_t[t] == sig_t[q] && t < q)) ++rk;
    if (rk < P.D) keep[rk] = q;
  }
  __syncthreads();
  const double smax = sig_t[keep[0]] > 0.0 ? sig_t[keep[0]] : 0.0;
  // new weights of the bond (kept values over the largest)
  __syncthreads();
  if (threadIdx.x < P.D) {
    const double s = sig_t[keep[threadIdx.x]];
    lam[(size_t)bd.k * P.D + threadIdx.x] = (smax > 0.0 && s > 0.0) ? s / smax : 0.0;
  }
  __syncthreads();
  // T_i = Q_i U: U[(c_i, S_i')][k] = Theta[:, keep k] / sigma_k
  su_scatter(P, si, Xi, lam, theta, [&](int c, int S, int kk) {
    const int q = keep[kk];
    const double s = sig_t[q];
    return s > 0.0 ? Th[(size_t)q * nt + c * 4 + S] / s : 0.0;
  });
  // T_j = Q_j V: V[(S_j', c_j)][k] = Vt[:, keep k] (zero where the value is 0)
  su_scatter(P, sj, Xj, lam, theta, [&](int c, int S, int kk) {
    const int q = keep[kk];
    return sig_t[q] > 0.0 ? Vt[(size_t)q * nt + S * n + c] : 0.0;
  });
}

// theta_out = theta with sqrt(lambda) on both ends of every bond.
__global__ void k_su_absorb(Prob P, const double* theta, const double* lam, double* out) {
  const int i = blockIdx.x;
  const int r = i / P.L2, c = i % P.L2;
  int dims[4];
  leg_dims(P, r, c, dims[0], dims[1], dims[2], dims[3]);
  const int bs = dims[0] * dims[1] * dims[2] * dims[3];
  const int po = param_offset(P, i);
  for (int idx = threadIdx.x; idx < P.d2 * bs; idx += blockDim.x) {
    int rem = idx % bs;
    int x[4];
    for (int l = 3; l >= 0; --l) {
      x[l] = rem % dims[l];
      rem /= dims[l];
    }
    double w = 1.0;
    for (int l = 0; l < 4; ++l) {
      const int k = leg_bond(P, r, c, l);
      if (k >= 0) w *= sqrt(lam[(size_t)k * P.D + x[l]]);
    }
    out[po + idx] = theta[po + idx] * w;
  }
}

size_t su_bond_doubles(const Prob& P) {
  const size_t n = (size_t)P.d2 * P.D, nt = 4 * n, m = (size_t)P.D * P.D * P.D;
  return 2 * m * n + 4 * n * n + 2 * nt * nt;
}

int su_max_group(const Prob& P) {
  int mx = 0;
  for (int g = 0; g < 4; ++g) mx = su_group_size(P, g) > mx ? su_group_size(P, g) : mx;
  return mx;
}

hipError_t launch_su_step(const Prob& P, double* theta, double* lam, double tau, double* ws, int32_t* status,
                          hipStream_t st) {
  const double et = exp(-tau * P.J1 / 4.0), es = exp(3.0 * tau * P.J1 / 4.0);
  const size_t stride = (su_bond_doubles(P) + 31) & ~(size_t)31;
  for (int g = 0; g < 4; ++g) {
    const int nb = su_group_size(P, g);
    if (nb == 0) continue;
    const int nt = 4 * P.d2 * P.D;
    const size_t lds = nt <= SU_LDS_NT ? 2 * (size_t)nt * nt * sizeof(double) : 0;
    hipLaunchKernelGGL(k_su_bond, dim3(nb), dim3(SU_NT), lds, st, P, g, theta, lam, et, es, ws, stride, status);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_su_absorb(const Prob& P, const double* theta, const double* lam, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_su_absorb, dim3(P.N), dim3(256), 0, st, P, theta, lam, out);
  return hipGetLastError();
}

}  // namespace peps
