// Workgroup-level strip contractions in FP64 (one workgroup = one chain).
//
// Index names: a / a2 = bonds of the top boundary MPS, b / b2 = bonds of the
// bottom boundary MPS, l / r = horizontal PEPS bonds, u / d = vertical PEPS
// legs.  Tensors are row-major in the order their names list the indices:
//   boundary tensors T[a][u][a2] (top) and B[b][d][b2] (bottom),
//   site slices W[l][u][r][d],
//   one-row environments E[a][l][b], two-row environments E[a][l1][l2][b].
// Every stage writes a full intermediate, then synchronises the workgroup.
#pragma once

#include "peps_common.hpp"

namespace peps {

struct Dim3 { int n0, n1, n2; };
struct Dim4 { int n0, n1, n2, n3; };

// One column of a one-row strip from the left:
//   out[a2][r][b2] = sum L[a][l][b] T[a][u][a2] W[l][u][r][d] B[b][d][b2]
__device__ inline void lstep1(double* out, const double* L, const double* T, Dim3 tD,
                              const double* W, Dim4 wD, const double* B, Dim3 bD,
                              double* X0, double* X1) {
  const int tid = threadIdx.x;
  const int na = tD.n0, nu = tD.n1, na2 = tD.n2;
  const int nl = wD.n0, nr = wD.n2, nd = wD.n3;
  const int nb = bD.n0, nb2 = bD.n2;
  // X0[l][b][u][a2] = sum_a L[a][l][b] T[a][u][a2]
  const int n0 = nl * nb * nu * na2;
  for (int idx = tid; idx < n0; idx += NT) {
    int a2 = idx % na2, t = idx / na2;
    int u = t % nu; t /= nu;
    int b = t % nb, l = t / nb;
    double s = 0.0;
    for (int a = 0; a < na; ++a) s += L[(a * nl + l) * nb + b] * T[(a * nu + u) * na2 + a2];
    X0[idx] = s;
  }
  __syncthreads();
  // X1[b][a2][r][d] = sum_{l,u} X0[l][b][u][a2] W[l][u][r][d]
  const int n1 = nb * na2 * nr * nd;
  for (int idx = tid; idx < n1; idx += NT) {
    int dd = idx % nd, t = idx / nd;
    int rr = t % nr; t /= nr;
    int a2 = t % na2, b = t / na2;
    double s = 0.0;
    for (int l = 0; l < nl; ++l)
      for (int u = 0; u < nu; ++u)
        s += X0[((l * nb + b) * nu + u) * na2 + a2] * W[((l * nu + u) * nr + rr) * nd + dd];
    X1[idx] = s;
  }
  __syncthreads();
  // out[a2][r][b2] = sum_{b,d} X1[b][a2][r][d] B[b][d][b2]
  const int n2 = na2 * nr * nb2;
  for (int idx = tid; idx < n2; idx += NT) {
    int b2 = idx % nb2, t = idx / nb2;
    int rr = t % nr, a2 = t / nr;
    double s = 0.0;
    for (int b = 0; b < nb; ++b)
      for (int dd = 0; dd < nd; ++dd)
        s += X1[((b * na2 + a2) * nr + rr) * nd + dd] * B[(b * nd + dd) * nb2 + b2];
    out[idx] = s;
  }
  __syncthreads();
}

// One column of a one-row strip from the right:
//   out[a][l][b] = sum T[a][u][a2] W[l][u][r][d] B[b][d][b2] R[a2][r][b2]
__device__ inline void rstep1(double* out, const double* R, const double* T, Dim3 tD,
                              const double* W, Dim4 wD, const double* B, Dim3 bD,
                              double* X0, double* X1) {
  const int tid = threadIdx.x;
  const int na = tD.n0, nu = tD.n1, na2 = tD.n2;
  const int nl = wD.n0, nr = wD.n2, nd = wD.n3;
  const int nb = bD.n0, nb2 = bD.n2;
  // X0[b][d][a2][r] = sum_b2 B[b][d][b2] R[a2][r][b2]
  const int n0 = nb * nd * na2 * nr;
  for (int idx = tid; idx < n0; idx += NT) {
    int rr = idx % nr, t = idx / nr;
    int a2 = t % na2; t /= na2;
    int dd = t % nd, b = t / nd;
    double s = 0.0;
    for (int b2 = 0; b2 < nb2; ++b2) s += B[(b * nd + dd) * nb2 + b2] * R[(a2 * nr + rr) * nb2 + b2];
    X0[idx] = s;
  }
  __syncthreads();
  // X1[l][u][b][a2] = sum_{r,d} W[l][u][r][d] X0[b][d][a2][r]
  const int n1 = nl * nu * nb * na2;
  for (int idx = tid; idx < n1; idx += NT) {
    int a2 = idx % na2, t = idx / na2;
    int b = t % nb; t /= nb;
    int u = t % nu, l = t / nu;
    double s = 0.0;
    for (int rr = 0; rr < nr; ++rr)
      for (int dd = 0; dd < nd; ++dd)
        s += W[((l * nu + u) * nr + rr) * nd + dd] * X0[((b * nd + dd) * na2 + a2) * nr + rr];
    X1[idx] = s;
  }
  __syncthreads();
  // out[a][l][b] = sum_{u,a2} T[a][u][a2] X1[l][u][b][a2]
  const int n2 = na * nl * nb;
  for (int idx = tid; idx < n2; idx += NT) {
    int b = idx % nb, t = idx / nb;
    int l = t % nl, a = t / nl;
    double s = 0.0;
    for (int u = 0; u < nu; ++u)
      for (int a2 = 0; a2 < na2; ++a2)
        s += T[(a * nu + u) * na2 + a2] * X1[((l * nu + u) * nb + b) * na2 + a2];
    out[idx] = s;
  }
  __syncthreads();
}

// One column of a two-row strip from the left:
//   out[a2][r1][r2][b2] = sum L[a][l1][l2][b] T[a][u][a2] W1[l1][u][r1][d1]
//                             W2[l2][d1][r2][d2] B[b][d2][b2]
__device__ inline void lstep2(double* out, const double* L, const double* T, Dim3 tD,
                              const double* W1, Dim4 w1, const double* W2, Dim4 w2,
                              const double* B, Dim3 bD, double* X0, double* X1) {
  const int tid = threadIdx.x;
  const int na = tD.n0, nu = tD.n1, na2 = tD.n2;
  const int nl1 = w1.n0, nr1 = w1.n2, nd1 = w1.n3;
  const int nl2 = w2.n0, nr2 = w2.n2, nd2 = w2.n3;
  const int nb = bD.n0, nb2 = bD.n2;
  // X0[l1][l2][b][u][a2] = sum_a L[a][l1][l2][b] T[a][u][a2]
  const int n0 = nl1 * nl2 * nb * nu * na2;
  for (int idx = tid; idx < n0; idx += NT) {
    int a2 = idx % na2, t = idx / na2;
    int u = t % nu; t /= nu;
    int b = t % nb; t /= nb;
    int l2 = t % nl2, l1 = t / nl2;
    double s = 0.0;
    for (int a = 0; a < na; ++a)
      s += L[((a * nl1 + l1) * nl2 + l2) * nb + b] * T[(a * nu + u) * na2 + a2];
    X0[idx] = s;
  }
  __syncthreads();
  // X1[l2][b][a2][r1][d1] = sum_{l1,u} X0[l1][l2][b][u][a2] W1[l1][u][r1][d1]
  const int n1 = nl2 * nb * na2 * nr1 * nd1;
  for (int idx = tid; idx < n1; idx += NT) {
    int d1 = idx % nd1, t = idx / nd1;
    int r1 = t % nr1; t /= nr1;
    int a2 = t % na2; t /= na2;
    int b = t % nb, l2 = t / nb;
    double s = 0.0;
    for (int l1 = 0; l1 < nl1; ++l1)
      for (int u = 0; u < nu; ++u)
        s += X0[(((l1 * nl2 + l2) * nb + b) * nu + u) * na2 + a2] * W1[((l1 * nu + u) * nr1 + r1) * nd1 + d1];
    X1[idx] = s;
  }
  __syncthreads();
  // X0[b][a2][r1][r2][d2] = sum_{l2,d1} X1[l2][b][a2][r1][d1] W2[l2][d1][r2][d2]
  const int n2 = nb * na2 * nr1 * nr2 * nd2;
  for (int idx = tid; idx < n2; idx += NT) {
    int d2 = idx % nd2, t = idx / nd2;
    int r2 = t % nr2; t /= nr2;
    int r1 = t % nr1; t /= nr1;
    int a2 = t % na2, b = t / na2;
    double s = 0.0;
    for (int l2 = 0; l2 < nl2; ++l2)
      for (int d1 = 0; d1 < nd1; ++d1)
        s += X1[(((l2 * nb + b) * na2 + a2) * nr1 + r1) * nd1 + d1] * W2[((l2 * nd1 + d1) * nr2 + r2) * nd2 + d2];
    X0[idx] = s;
  }
  __syncthreads();
  // out[a2][r1][r2][b2] = sum_{b,d2} X0[b][a2][r1][r2][d2] B[b][d2][b2]
  const int n3 = na2 * nr1 * nr2 * nb2;
  for (int idx = tid; idx < n3; idx += NT) {
    int b2 = idx % nb2, t = idx / nb2;
    int r2 = t % nr2; t /= nr2;
    int r1 = t % nr1, a2 = t / nr1;
    double s = 0.0;
    for (int b = 0; b < nb; ++b)
      for (int d2 = 0; d2 < nd2; ++d2)
        s += X0[(((b * na2 + a2) * nr1 + r1) * nr2 + r2) * nd2 + d2] * B[(b * nd2 + d2) * nb2 + b2];
    out[idx] = s;
  }
  __syncthreads();
}

// One column of a two-row strip from the right:
//   out[a][l1][l2][b] = sum T[a][u][a2] W1[l1][u][r1][d1] W2[l2][d1][r2][d2]
//                           B[b][d2][b2] R[a2][r1][r2][b2]
__device__ inline void rstep2(double* out, const double* R, const double* T, Dim3 tD,
                              const double* W1, Dim4 w1, const double* W2, Dim4 w2,
                              const double* B, Dim3 bD, double* X0, double* X1) {
  const int tid = threadIdx.x;
  const int na = tD.n0, nu = tD.n1, na2 = tD.n2;
  const int nl1 = w1.n0, nr1 = w1.n2, nd1 = w1.n3;
  const int nl2 = w2.n0, nr2 = w2.n2, nd2 = w2.n3;
  const int nb = bD.n0, nb2 = bD.n2;
  // X0[b][d2][a2][r1][r2] = sum_b2 B[b][d2][b2] R[a2][r1][r2][b2]
  const int n0 = nb * nd2 * na2 * nr1 * nr2;
  for (int idx = tid; idx < n0; idx += NT) {
    int r2 = idx % nr2, t = idx / nr2;
    int r1 = t % nr1; t /= nr1;
    int a2 = t % na2; t /= na2;
    int d2 = t % nd2, b = t / nd2;
    double s = 0.0;
    for (int b2 = 0; b2 < nb2; ++b2)
      s += B[(b * nd2 + d2) * nb2 + b2] * R[((a2 * nr1 + r1) * nr2 + r2) * nb2 + b2];
    X0[idx] = s;
  }
  __syncthreads();
  // X1[l2][d1][b][a2][r1] = sum_{r2,d2} W2[l2][d1][r2][d2] X0[b][d2][a2][r1][r2]
  const int n1 = nl2 * nd1 * nb * na2 * nr1;
  for (int idx = tid; idx < n1; idx += NT) {
    int r1 = idx % nr1, t = idx / nr1;
    int a2 = t % na2; t /= na2;
    int b = t % nb; t /= nb;
    int d1 = t % nd1, l2 = t / nd1;
    double s = 0.0;
    for (int r2 = 0; r2 < nr2; ++r2)
      for (int d2 = 0; d2 < nd2; ++d2)
        s += W2[((l2 * nd1 + d1) * nr2 + r2) * nd2 + d2] * X0[(((b * nd2 + d2) * na2 + a2) * nr1 + r1) * nr2 + r2];
    X1[idx] = s;
  }
  __syncthreads();
  // X0[l1][u][l2][b][a2] = sum_{r1,d1} W1[l1][u][r1][d1] X1[l2][d1][b][a2][r1]
  const int n2 = nl1 * nu * nl2 * nb * na2;
  for (int idx = tid; idx < n2; idx += NT) {
    int a2 = idx % na2, t = idx / na2;
    int b = t % nb; t /= nb;
    int l2 = t % nl2; t /= nl2;
    int u = t % nu, l1 = t / nu;
    double s = 0.0;
    for (int r1 = 0; r1 < nr1; ++r1)
      for (int d1 = 0; d1 < nd1; ++d1)
        s += W1[((l1 * nu + u) * nr1 + r1) * nd1 + d1] * X1[(((l2 * nd1 + d1) * nb + b) * na2 + a2) * nr1 + r1];
    X0[idx] = s;
  }
  __syncthreads();
  // out[a][l1][l2][b] = sum_{u,a2} T[a][u][a2] X0[l1][u][l2][b][a2]
  const int n3 = na * nl1 * nl2 * nb;
  for (int idx = tid; idx < n3; idx += NT) {
    int b = idx % nb, t = idx / nb;
    int l2 = t % nl2; t /= nl2;
    int l1 = t % nl1, a = t / nl1;
    double s = 0.0;
    for (int u = 0; u < nu; ++u)
      for (int a2 = 0; a2 < na2; ++a2)
        s += T[(a * nu + u) * na2 + a2] * X0[(((l1 * nu + u) * nl2 + l2) * nb + b) * na2 + a2];
    out[idx] = s;
  }
  __syncthreads();
}

// Environment of one site in a one-row strip (the strip is linear in W):
//   env[l][u][r][d] = sum L[a][l][b] T[a][u][a2] B[b][d][b2] R[a2][r][b2]
__device__ inline void site_env1(double* env, const double* L, const double* T, Dim3 tD,
                                 const double* B, Dim3 bD, const double* R, int nl, int nr,
                                 double* X0, double* X1) {
  const int tid = threadIdx.x;
  const int na = tD.n0, nu = tD.n1, na2 = tD.n2;
  const int nb = bD.n0, nd = bD.n1, nb2 = bD.n2;
  // X0[l][b][u][a2] = sum_a L[a][l][b] T[a][u][a2]
  const int n0 = nl * nb * nu * na2;
  for (int idx = tid; idx < n0; idx += NT) {
    int a2 = idx % na2, t = idx / na2;
    int u = t % nu; t /= nu;
    int b = t % nb, l = t / nb;
    double s = 0.0;
    for (int a = 0; a < na; ++a) s += L[(a * nl + l) * nb + b] * T[(a * nu + u) * na2 + a2];
    X0[idx] = s;
  }
  __syncthreads();
  // X1[l][u][a2][d][b2] = sum_b X0[l][b][u][a2] B[b][d][b2]
  const int n1 = nl * nu * na2 * nd * nb2;
  for (int idx = tid; idx < n1; idx += NT) {
    int b2 = idx % nb2, t = idx / nb2;
    int dd = t % nd; t /= nd;
    int a2 = t % na2; t /= na2;
    int u = t % nu, l = t / nu;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += X0[((l * nb + b) * nu + u) * na2 + a2] * B[(b * nd + dd) * nb2 + b2];
    X1[idx] = s;
  }
  __syncthreads();
  // env[l][u][r][d] = sum_{a2,b2} X1[l][u][a2][d][b2] R[a2][r][b2]
  const int n2 = nl * nu * nr * nd;
  for (int idx = tid; idx < n2; idx += NT) {
    int dd = idx % nd, t = idx / nd;
    int rr = t % nr; t /= nr;
    int u = t % nu, l = t / nu;
    double s = 0.0;
    for (int a2 = 0; a2 < na2; ++a2)
      for (int b2 = 0; b2 < nb2; ++b2)
        s += X1[(((l * nu + u) * na2 + a2) * nd + dd) * nb2 + b2] * R[(a2 * nr + rr) * nb2 + b2];
    env[idx] = s;
  }
  __syncthreads();
}

// sum_i x[i] y[i], identical on every thread.
__device__ inline double wg_dot(const double* x, const double* y, int n, double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s += x[i] * y[i];
  return wg_sum(s, red);
}

}  // namespace peps
