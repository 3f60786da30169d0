// Workgroup-level strip contractions (one workgroup = one chain), each a
// chain of small GEMMs on MFMA 16x16x4 tiles.
//
// Index names: a / a2 = bonds of the top boundary MPS, b / b2 = bonds of the
// bottom boundary MPS, l / r = horizontal PEPS bonds, u / d = vertical PEPS
// legs.  Tensors are row-major in the order their names list the indices:
//   boundary tensors T[a][u][a2] (top) and B[b][d][b2] (bottom),
//   site slices W[l][u][r][d],
//   one-row environments E[a][l][b], two-row environments E[a][l1][l2][b].
// Every stage C = A B is a GEMM whose operands are addressed through
// two-level index maps (a fused index i = (i1, i2) maps to i1 s1 + i2 s2),
// so no operand is ever permuted in memory.  Stages are separated by a
// workgroup barrier; intermediates live in the chain's workspace.
//
// The last stage of every step can scale its output by an exact power of two
// and record the largest magnitude it wrote (one value per wave), which the
// FP32 form uses to keep environments in range: the caller carries the
// exponents in integers and applies them to the FP64 ratios.
#pragma once

#include "peps_common.hpp"

namespace peps {

struct Dim3 { int n0, n1, n2; };
struct Dim4 { int n0, n1, n2, n3; };

// i -> (i / n2) * s1 + (i % n2) * s2
struct Map2 {
  int n2, s1, s2;
  __device__ inline int operator()(int i) const { return (i / n2) * s1 + (i % n2) * s2; }
};
__device__ inline Map2 mstride(int s) { return Map2{1, s, 0}; }   // i -> i * s
__device__ inline Map2 mid() { return Map2{1, 1, 0}; }            // i -> i

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// MFMA 16x16x4: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator register v of lane l holds C[row(l, v)][l % 16].
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  using acc = f64x4;
  __device__ static inline acc run(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static inline int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <> struct Mfma<float> {
  using acc = f32x4;
  __device__ static inline acc run(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static inline int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// Whether a k-map is unit-stride inside every aligned group of four indices
// (offset(4g + u) = offset(4g) + u) with offset(4g) a multiple of 4, and
// whether a row / column map gives multiples of 4 only.
__device__ inline bool map_unit4(Map2 mk) {
  return (mk.n2 == 1 && mk.s1 == 1) || (mk.n2 % 4 == 0 && mk.s2 == 1 && mk.s1 % 4 == 0);
}
__device__ inline bool map_mult4(Map2 mm) { return mm.s1 % 4 == 0 && (mm.n2 == 1 || mm.s2 % 4 == 0); }

// C(m, n) = sum_k A(m, k) B(k, n) for m < M, n < N, k < K, with
//   A(m, k) = A[am(m) + ak(k)], B(k, n) = B[bk(k) + bn(n)], C at cm(m) + cn(n).
// Tiles of 16 x 16 are dealt round-robin to the waves of the workgroup.
// The stored value is the accumulator times `osc`; when `wmax` is given,
// wave w writes the largest stored magnitude of its tiles to wmax[w].
// Ends with a workgroup barrier.
//
// When an operand's k-map is unit-stride in aligned groups of four (and K
// is a multiple of 4), lane group q (lanes 16q..16q+15) takes, inside each
// block of 16 k, the four consecutive indices 16 j + 4 q + u (u = 0..3, one
// per MFMA step), so that operand is read with one vector load per lane
// instead of four scalar ones: the address unit, which the gathers keep
// busy, then handles a quarter of the load instructions for it.  Otherwise
// step u takes 16 j + 4 u + q, which keeps the four lane groups of a
// scalar load on neighbouring k.
template <typename T>
__device__ inline void wg_gemm(T* C, Map2 cm, Map2 cn, const T* A, Map2 am, Map2 ak, const T* B, Map2 bk, Map2 bn,
                               int M, int N, int K, T osc = T(1), float* wmax = nullptr) {
  using MF = Mfma<T>;
  typedef T V4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
  constexpr uintptr_t VAL = 4 * sizeof(T) - 1;
  const bool vecA = (K & 3) == 0 && map_unit4(ak) && map_mult4(am) && ((uintptr_t)A & VAL) == 0;
  const bool vecB = (K & 3) == 0 && map_unit4(bk) && map_mult4(bn) && ((uintptr_t)B & VAL) == 0;
  const bool grouped = vecA || vecB;
  float mx = 0.0f;
  for (int t = wave; t < tm * tn; t += nw) {
    const int m0 = (t / tn) << 4, n0 = (t % tn) << 4;
    const int m = m0 + li, n = n0 + li;
    const bool mv = m < M, nv = n < N;
    const int ao = mv ? am(m) : 0, bo = nv ? bn(n) : 0;
    typename MF::acc c = {0, 0, 0, 0};
    for (int k0 = 0; k0 < K; k0 += 16) {
      const int kg = k0 + 4 * lk;   // this lane group's four k (grouped order)
      T a[4], b[4];
      // all operand loads of the block are issued before its first MFMA
      if (vecA) {
        const bool ok = mv && kg < K;
        const V4 v = *(const V4*)(A + (ok ? ao + ak(kg) : 0));   // A[0..3] exist: K >= 4
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = ok ? v[u] : T(0);
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = grouped ? kg + u : k0 + 4 * u + lk;
          a[u] = (mv && k < K) ? A[ao + ak(k)] : T(0);
        }
      }
      if (vecB) {
        const bool ok = nv && kg < K;
        const V4 v = *(const V4*)(B + (ok ? bo + bk(kg) : 0));
#pragma unroll
        for (int u = 0; u < 4; ++u) b[u] = ok ? v[u] : T(0);
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = grouped ? kg + u : k0 + 4 * u + lk;
          b[u] = (nv && k < K) ? B[bk(k) + bo] : T(0);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) c = MF::run(a[u], b[u], c);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = m0 + MF::row(lane, v);
      const T val = c[v] * osc;
      if (row < M && nv) {
        C[cm(row) + cn(n)] = val;
        mx = fmaxf(mx, fabsf((float)val));
      }
    }
  }
  if (wmax) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (lane == 0) wmax[wave] = mx;
  }
  __syncthreads();
}

template <typename T>
__device__ inline void wg_gemm_rm(T* C, const T* A, Map2 am, Map2 ak, const T* B, Map2 bk, Map2 bn, int M, int N,
                                  int K, T osc = T(1), float* wmax = nullptr) {
  wg_gemm<T>(C, mstride(N), mid(), A, am, ak, B, bk, bn, M, N, K, osc, wmax);
}

// One column of a one-row strip from the left:
//   out[a2][r][b2] = sum L[a][l][b] T[a][u][a2] W[l][u][r][d] B[b][d][b2]
template <typename T>
__device__ inline void lstep1(T* out, const T* L, const T* Tt, Dim3 tD, const T* W, Dim4 wD, const T* B, Dim3 bD,
                              T* X0, T* X1, T osc = T(1), float* wmax = nullptr) {
  const int na = tD.n0, nu = tD.n1, na2 = tD.n2;
  const int nl = wD.n0, nr = wD.n2, nd = wD.n3;
  const int nb = bD.n0, nb2 = bD.n2;
  // X0[(l b)][(u a2)] = sum_a L[a][(l b)] T[a][(u a2)]
  wg_gemm_rm<T>(X0, L, mid(), mstride(nl * nb), Tt, mstride(nu * na2), mid(), nl * nb, nu * na2, na);
  // X1[(b a2)][(r d)] = sum_{l,u} X0[l][b][u][a2] W[(l u)][(r d)]
  wg_gemm_rm<T>(X1, X0, Map2{na2, nu * na2, 1}, Map2{nu, nb * nu * na2, na2}, W, mstride(nr * nd), mid(),
                nb * na2, nr * nd, nl * nu);
  // out[(a2 r)][b2] = sum_{b,d} X1[b][a2][r][d] B[(b d)][b2]
  wg_gemm_rm<T>(out, X1, mstride(nd), Map2{nd, na2 * nr * nd, 1}, B, mstride(nb2), mid(), na2 * nr, nb2, nb * nd, osc, wmax);
}

// One column of a one-row strip from the right:
//   out[a][l][b] = sum T[a][u][a2] W[l][u][r][d] B[b][d][b2] R[a2][r][b2]
template <typename T>
__device__ inline void rstep1(T* out, const T* R, const T* Tt, Dim3 tD, const T* W, Dim4 wD, const T* B, Dim3 bD,
                              T* X0, T* X1, T osc = T(1), float* wmax = nullptr) {
  const int na = tD.n0, nu = tD.n1, na2 = tD.n2;
  const int nl = wD.n0, nr = wD.n2, nd = wD.n3;
  const int nb = bD.n0, nb2 = bD.n2;
  // X0[(b d)][(a2 r)] = sum_b2 B[(b d)][b2] R[(a2 r)][b2]
  wg_gemm_rm<T>(X0, B, mstride(nb2), mid(), R, mid(), mstride(nb2), nb * nd, na2 * nr, nb2);
  // X1[(l u)][(b a2)] = sum_{r,d} W[(l u)][(r d)] X0[b][d][a2][r]
  wg_gemm_rm<T>(X1, W, mstride(nr * nd), mid(), X0, Map2{nd, 1, na2 * nr}, Map2{na2, nd * na2 * nr, nr}, nl * nu,
                nb * na2, nr * nd);
  // out[a][(l b)] = sum_{u,a2} T[a][(u a2)] X1[l][u][b][a2]
  wg_gemm_rm<T>(out, Tt, mstride(nu * na2), mid(), X1, Map2{na2, nb * na2, 1}, Map2{nb, nu * nb * na2, na2}, na,
                nl * nb, nu * na2, osc, wmax);
}

// One column of a two-row strip from the left:
//   out[a2][r1][r2][b2] = sum L[a][l1][l2][b] T[a][u][a2] W1[l1][u][r1][d1]
//                             W2[l2][d1][r2][d2] B[b][d2][b2]
template <typename T>
__device__ inline void lstep2(T* out, const T* L, const T* Tt, Dim3 tD, const T* W1, Dim4 w1, const T* W2, Dim4 w2,
                              const T* B, Dim3 bD, T* X0, T* X1, T osc = T(1), float* wmax = nullptr) {
  const int na = tD.n0, nu = tD.n1, na2 = tD.n2;
  const int nl1 = w1.n0, nr1 = w1.n2, nd1 = w1.n3;
  const int nl2 = w2.n0, nr2 = w2.n2, nd2 = w2.n3;
  const int nb = bD.n0, nb2 = bD.n2;
  // X0[(l1 l2 b)][(u a2)] = sum_a L[a][(l1 l2 b)] T[a][(u a2)]
  wg_gemm_rm<T>(X0, L, mid(), mstride(nl1 * nl2 * nb), Tt, mstride(nu * na2), mid(), nl1 * nl2 * nb, nu * na2, na);
  // X1[(l2 b a2)][(r1 d1)] = sum_{l1,u} X0[l1][(l2 b)][u][a2] W1[(l1 u)][(r1 d1)]
  wg_gemm_rm<T>(X1, X0, Map2{na2, nu * na2, 1}, Map2{nu, nl2 * nb * nu * na2, na2}, W1, mstride(nr1 * nd1), mid(),
                nl2 * nb * na2, nr1 * nd1, nl1 * nu);
  // X0[(b a2 r1)][(r2 d2)] = sum_{l2,d1} X1[l2][(b a2 r1)][d1] W2[(l2 d1)][(r2 d2)]
  wg_gemm_rm<T>(X0, X1, mstride(nd1), Map2{nd1, nb * na2 * nr1 * nd1, 1}, W2, mstride(nr2 * nd2), mid(),
                nb * na2 * nr1, nr2 * nd2, nl2 * nd1);
  // out[(a2 r1 r2)][b2] = sum_{b,d2} X0[b][(a2 r1 r2)][d2] B[(b d2)][b2]
  wg_gemm_rm<T>(out, X0, mstride(nd2), Map2{nd2, na2 * nr1 * nr2 * nd2, 1}, B, mstride(nb2), mid(),
                na2 * nr1 * nr2, nb2, nb * nd2, osc, wmax);
}

// One column of a two-row strip from the right:
//   out[a][l1][l2][b] = sum T[a][u][a2] W1[l1][u][r1][d1] W2[l2][d1][r2][d2]
//                           B[b][d2][b2] R[a2][r1][r2][b2]
template <typename T>
__device__ inline void rstep2(T* out, const T* R, const T* Tt, Dim3 tD, const T* W1, Dim4 w1, const T* W2, Dim4 w2,
                              const T* B, Dim3 bD, T* X0, T* X1, T osc = T(1), float* wmax = nullptr) {
  const int na = tD.n0, nu = tD.n1, na2 = tD.n2;
  const int nl1 = w1.n0, nr1 = w1.n2, nd1 = w1.n3;
  const int nl2 = w2.n0, nr2 = w2.n2, nd2 = w2.n3;
  const int nb = bD.n0, nb2 = bD.n2;
  // X0[(b d2)][(a2 r1 r2)] = sum_b2 B[(b d2)][b2] R[(a2 r1 r2)][b2]
  wg_gemm_rm<T>(X0, B, mstride(nb2), mid(), R, mid(), mstride(nb2), nb * nd2, na2 * nr1 * nr2, nb2);
  // X1[(l2 d1)][(b a2 r1)] = sum_{r2,d2} W2[(l2 d1)][(r2 d2)] X0[b][d2][(a2 r1)][r2]
  wg_gemm_rm<T>(X1, W2, mstride(nr2 * nd2), mid(), X0, Map2{nd2, 1, na2 * nr1 * nr2},
                Map2{na2 * nr1, nd2 * na2 * nr1 * nr2, nr2}, nl2 * nd1, nb * na2 * nr1, nr2 * nd2);
  // X0[(l1 u)][(l2 b a2)] = sum_{r1,d1} W1[(l1 u)][(r1 d1)] X1[l2][d1][(b a2)][r1]
  wg_gemm_rm<T>(X0, W1, mstride(nr1 * nd1), mid(), X1, Map2{nd1, 1, nb * na2 * nr1},
                Map2{nb * na2, nd1 * nb * na2 * nr1, nr1}, nl1 * nu, nl2 * nb * na2, nr1 * nd1);
  // out[a][(l1 l2 b)] = sum_{u,a2} T[a][(u a2)] X0[l1][u][(l2 b)][a2]
  wg_gemm_rm<T>(out, Tt, mstride(nu * na2), mid(), X0, Map2{na2, nl2 * nb * na2, 1},
                Map2{nl2 * nb, nu * nl2 * nb * na2, na2}, na, nl1 * nl2 * nb, nu * na2, osc, wmax);
}

// Environment of one site in a one-row strip (the strip is linear in W):
//   env[l][u][r][d] = osc * sum L[a][l][b] T[a][u][a2] B[b][d][b2] R[a2][r][b2]
template <typename T>
__device__ inline void site_env1(T* env, const T* L, const T* Tt, Dim3 tD, const T* B, Dim3 bD, const T* R, int nl,
                                 int nr, T* X0, T* X1, T osc = T(1)) {
  const int na = tD.n0, nu = tD.n1, na2 = tD.n2;
  const int nb = bD.n0, nd = bD.n1, nb2 = bD.n2;
  // X0[(l b)][(u a2)] = sum_a L[a][(l b)] T[a][(u a2)]
  wg_gemm_rm<T>(X0, L, mid(), mstride(nl * nb), Tt, mstride(nu * na2), mid(), nl * nb, nu * na2, na);
  // X1[(l u a2)][(d b2)] = sum_b X0[l][b][(u a2)] B[b][(d b2)]
  wg_gemm_rm<T>(X1, X0, Map2{nu * na2, nb * nu * na2, 1}, mstride(nu * na2), B, mstride(nd * nb2), mid(),
                nl * nu * na2, nd * nb2, nb);
  // env[(l u)][r][d] = sum_{a2,b2} X1[(l u)][a2][d][b2] R[a2][r][b2]   (rows (l u d), cols r)
  wg_gemm<T>(env, Map2{nd, nr * nd, 1}, mstride(nd), X1, Map2{nd, na2 * nd * nb2, nb2}, Map2{nb2, nd * nb2, 1}, R,
             Map2{nb2, nr * nb2, 1}, mstride(nb2), nl * nu * nd, nr, na2 * nb2, osc);
}

// sum_i x[i] y[i], identical on every thread.
template <typename T>
__device__ inline double wg_dot(const T* x, const T* y, int n, double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s += (double)x[i] * (double)y[i];
  return wg_sum(s, red);
}

}  // namespace peps
