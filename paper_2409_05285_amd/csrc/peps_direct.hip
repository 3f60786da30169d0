// Direct (autoregressive) sampling of the vectorised PEPS (Appendix A,
// Eqs. A2-A7): each chain draws its configuration site by site, row-major,
// from the conditional probabilities of the double-layer network
// sum_S rho(S)^2, with the rows already drawn entering as their single-layer
// top boundary paired with itself.
//
// Layout of the double layer.  Site tensors E_i = sum_S T_i[S] (x) T_i[S]
// with every leg a pair (x, x') of dimension D^2, x' fastest; they form a
// PEPS with one physical digit (d^2 = 1), so its bottom boundaries come from
// the same row compression as the single-layer ones, run on one "chain"
// whose parameter vector is the E tensors.  The top of the rows already
// drawn is top (x) top, materialised per row; the site whose conditional is
// wanted is closed by its environment (site_env1), and the d^2 candidate
// weights are quadratic forms of that environment in the slice T_i[x].
//
// One workgroup per chain for a whole row: the right environments of the
// row (double-layer tensors only), then a left-to-right pass that draws one
// site at a time, absorbing the pair tensor of the drawn digit.  Between
// rows the single-layer top boundary of every chain is compressed by the
// usual row kernel on the drawn digits.
#include <math.h>

#include "peps_chain.hpp"
#include "peps_common.hpp"
#include "peps_contract.hpp"
#include "peps_kernels.hpp"

namespace peps {

namespace {

constexpr int MAX_D2 = 16;

// Quadratic forms q(x) = sum_{i,j} env[pair(i,j)] T_x[i] T_x[j] for every
// digit x, env indexed [(l l')][(u u')][(r r')][(d d')] over the site's leg
// dimensions; same bits on every thread.
__device__ void site_weights(const Prob& P, const Geo& g, const double* theta, int r, int c, const double* env,
                             double* q, double* red) {
  const Dim4 w = wdim(P, r, c);
  const int bs = w.n0 * w.n1 * w.n2 * w.n3;
  const double* T0 = theta + g.poff[r * P.L2 + c];
  double acc[MAX_D2];
#pragma unroll
  for (int x = 0; x < MAX_D2; ++x) acc[x] = 0.0;
  const int nu2 = w.n1 * w.n1, nr2 = w.n2 * w.n2, nd2 = w.n3 * w.n3;
  for (int e = threadIdx.x; e < bs * bs; e += NT) {
    int t = e;
    const int dq = t % nd2; t /= nd2;
    const int rq = t % nr2; t /= nr2;
    const int uq = t % nu2; t /= nu2;
    const int lq = t;
    const int i = ((lq / w.n0 * w.n1 + uq / w.n1) * w.n2 + rq / w.n2) * w.n3 + dq / w.n3;
    const int j = ((lq % w.n0 * w.n1 + uq % w.n1) * w.n2 + rq % w.n2) * w.n3 + dq % w.n3;
    const double ev = env[e];
#pragma unroll
    for (int x = 0; x < MAX_D2; ++x)
      if (x < P.d2) acc[x] += ev * T0[(size_t)x * bs + i] * T0[(size_t)x * bs + j];
  }
  for (int x = 0; x < P.d2; ++x) {
    const double s = wg_sum(acc[x], red);
    if (threadIdx.x == 0) q[x] = s;
  }
  __syncthreads();
}

// P(x) = T_x (x) T_x in the layout of the double-layer site tensors.
__device__ void pair_slice(const Prob& P, const Geo& g, const double* theta, int r, int c, int x, double* out) {
  const Dim4 w = wdim(P, r, c);
  const int bs = w.n0 * w.n1 * w.n2 * w.n3;
  const double* Tx = theta + g.poff[r * P.L2 + c] + (size_t)x * bs;
  const int nu2 = w.n1 * w.n1, nr2 = w.n2 * w.n2, nd2 = w.n3 * w.n3;
  for (int e = threadIdx.x; e < bs * bs; e += NT) {
    int t = e;
    const int dq = t % nd2; t /= nd2;
    const int rq = t % nr2; t /= nr2;
    const int uq = t % nu2; t /= nu2;
    const int lq = t;
    const int i = ((lq / w.n0 * w.n1 + uq / w.n1) * w.n2 + rq / w.n2) * w.n3 + dq / w.n3;
    const int j = ((lq % w.n0 * w.n1 + uq % w.n1) * w.n2 + rq % w.n2) * w.n3 + dq % w.n3;
    out[e] = Tx[i] * Tx[j];
  }
  __syncthreads();
}

// E_i = sum_S T_i[S] (x) T_i[S], one workgroup per site; also clears the
// one-chain configuration of the double layer (all digits 0).
__global__ void __launch_bounds__(NT) k_double_layer(Prob P, Prob Q, const double* theta, double* eth,
                                                      uint8_t* cfg_q) {
  __shared__ Geo g, gq;
  if (threadIdx.x == 0) {
    build_geo(P, g);
    build_geo(Q, gq);
  }
  __syncthreads();
  const int site = blockIdx.x, r = site / P.L2, c = site % P.L2;
  const Dim4 w = wdim(P, r, c);
  const int bs = w.n0 * w.n1 * w.n2 * w.n3;
  const double* T0 = theta + g.poff[site];
  double* E = eth + gq.poff[site];
  const int nu2 = w.n1 * w.n1, nr2 = w.n2 * w.n2, nd2 = w.n3 * w.n3;
  for (int e = threadIdx.x; e < bs * bs; e += NT) {
    int t = e;
    const int dq = t % nd2; t /= nd2;
    const int rq = t % nr2; t /= nr2;
    const int uq = t % nu2; t /= nu2;
    const int lq = t;
    const int i = ((lq / w.n0 * w.n1 + uq / w.n1) * w.n2 + rq / w.n2) * w.n3 + dq / w.n3;
    const int j = ((lq % w.n0 * w.n1 + uq % w.n1) * w.n2 + rq % w.n2) * w.n3 + dq % w.n3;
    double s = 0.0;
    for (int x = 0; x < P.d2; ++x) s += T0[(size_t)x * bs + i] * T0[(size_t)x * bs + j];
    E[e] = s;
  }
  if (threadIdx.x == 0) cfg_q[site] = 0;
}

// One row of every chain's draw.  dws: per-chain scratch of stride
// L.stride doubles; wsq: the double layer's one-chain workspace.
__global__ void __launch_bounds__(NT) k_direct_row(Prob P, Prob Q, DirectLayout DL, const double* theta,
                                                    const double* eth, uint8_t* configs, double* ws,
                                                    const double* wsq, double* dws, int r, uint64_t seed,
                                                    uint64_t draw, int reweight, const double* b_diag,
                                                    double* log_p, int32_t* status) {
  __shared__ Geo g, gq;
  __shared__ double red[NT];
  __shared__ double q[MAX_D2];
  __shared__ int pick_s;
  __shared__ Dim3 tdD[MAX_L], bqD[MAX_L];
  __shared__ const double* Bq[MAX_L];
  __shared__ double one;
  const int tid = threadIdx.x, ch = blockIdx.x;
  uint8_t* S = configs + (size_t)ch * P.N;
  double lp = r == 0 ? 0.0 : log_p[ch];
  if (!(lp > -INFINITY)) return;   // an earlier row failed (same value on every thread)
  const ChainWS w = chain_ws(P, ws, ch);
  const ChainWS wq = chain_ws(Q, (double*)wsq, 0);
  double* base = dws + (size_t)ch * DL.stride;
  double* TD = base + DL.off_td;
  double* R = base + DL.off_R;
  double* Lb = base + DL.off_L;
  double* X0 = base + DL.off_X0;
  double* X1 = base + DL.off_X1;
  double* env = base + DL.off_env;
  double* Px = base + DL.off_Px;
  if (tid == 0) {
    build_geo(P, g);
    build_geo(Q, gq);
    one = 1.0;
    for (int c = 0; c < P.L2; ++c) {
      if (r >= 1) {
        const int a = g.ba[0][r - 1][c], b = g.bb[0][r - 1][c];
        tdD[c] = Dim3{a * a, P.D * P.D, b * b};
      } else {
        tdD[c] = Dim3{1, 1, 1};
      }
      if (r + 1 <= P.L1 - 1) {
        Bq[c] = wq.bot + ((size_t)(r + 1) * P.L2 + c) * Q.TS;
        bqD[c] = Dim3{gq.ba[1][r + 1][c], Q.D, gq.bb[1][r + 1][c]};
      } else {
        Bq[c] = &one;
        bqD[c] = Dim3{1, 1, 1};
      }
    }
  }
  __syncthreads();
  // the drawn rows' top boundary paired with itself: [(a a')][(u u')][(b b')]
  for (int c = 0; c < P.L2; ++c) {
    double* td = TD + (size_t)c * DL.TDS;
    if (r == 0) {
      if (tid == 0) td[0] = 1.0;
      continue;
    }
    const int a = g.ba[0][r - 1][c], b = g.bb[0][r - 1][c], u = P.D;
    const double* t = w.top + ((size_t)(r - 1) * P.L2 + c) * P.TS;
    const int n = a * a * u * u * b * b;
    for (int e = tid; e < n; e += NT) {
      int k = e;
      const int bq = k % (b * b); k /= b * b;
      const int uq = k % (u * u); k /= u * u;
      const int aq = k;
      td[e] = t[((aq / a) * u + uq / u) * b + bq / b] * t[((aq % a) * u + uq % u) * b + bq % b];
    }
  }
  __syncthreads();
  // right environments R_c of the row's double layer, R_{L2} = 1
  if (tid == 0) R[(size_t)P.L2 * DL.ENV] = 1.0;
  __syncthreads();
  for (int c = P.L2 - 1; c >= 1; --c) {
    const double* E = eth + gq.poff[r * P.L2 + c];
    rstep1<double>(R + (size_t)c * DL.ENV, R + (size_t)(c + 1) * DL.ENV, TD + (size_t)c * DL.TDS, tdD[c], E,
                   wdim(Q, r, c), Bq[c], bqD[c], X0, X1);
  }
  // left-to-right draws
  double* Lc = Lb;
  double* Ln = Lb + DL.ENV;
  if (tid == 0) Lc[0] = 1.0;
  __syncthreads();
  const double bd = reweight ? b_diag[0] : 1.0;
  for (int c = 0; c < P.L2; ++c) {
    const Dim4 wq4 = wdim(Q, r, c);
    site_env1<double>(env, Lc, TD + (size_t)c * DL.TDS, tdD[c], Bq[c], bqD[c], R + (size_t)(c + 1) * DL.ENV,
                      wq4.n0, wq4.n2, X0, X1);
    site_weights(P, g, theta, r, c, env, q, red);
    const int i = r * P.L2 + c;
    if (tid == 0) {
      double p[MAX_D2];
      double tot = 0.0;
      for (int x = 0; x < P.d2; ++x) {
        p[x] = q[x] > 0.0 ? q[x] : 0.0;
        tot += p[x];
      }
      int x_pick = -1;
      bool ok = tot > 0.0 && isfinite(tot);
      if (ok) {
        for (int x = 0; x < P.d2; ++x) p[x] /= tot;
        if (reweight) {
          double s = 0.0;
          for (int x = 0; x < P.d2; ++x) {
            p[x] = (ket_of(P, x) != bra_of(P, x) ? 1.0 : bd) * sqrt(p[x]);
            s += p[x];
          }
          ok = s > 0.0 && isfinite(s);   // false when b = 0 leaves no digit
          if (ok)
            for (int x = 0; x < P.d2; ++x) p[x] /= s;
        }
      }
      if (ok) {
        const U64x4 rw = philox4x64_10((uint64_t)ch, draw, (uint64_t)i, 3ull, seed, 0ull);
        const double u = (double)(rw.v[0] >> 11) * 0x1.0p-53;
        double cum = 0.0;
        int last = 0;
        for (int x = 0; x < P.d2; ++x) {
          if (p[x] > 0.0) last = x;
          cum += p[x];
          if (x_pick < 0 && u < cum) x_pick = x;
        }
        if (x_pick < 0) x_pick = last;
        lp += log(p[x_pick]);
        S[i] = (uint8_t)x_pick;
      } else {
        set_status(status, isfinite(tot) && isfinite(bd) ? PEPS_ERR_ZERO_AMPLITUDE : PEPS_ERR_NONFINITE);
        lp = -INFINITY;
        for (int k = i; k < P.N; ++k) S[k] = 0;
      }
      pick_s = x_pick;
    }
    __syncthreads();
    const int x = pick_s;
    if (x < 0) break;
    if (c + 1 < P.L2) {
      pair_slice(P, g, theta, r, c, x, Px);
      lstep1<double>(Ln, Lc, TD + (size_t)c * DL.TDS, tdD[c], Px, wq4, Bq[c], bqD[c], X0, X1);
      double* t = Lc;
      Lc = Ln;
      Ln = t;
    }
  }
  if (tid == 0) log_p[ch] = lp;
}

// b_diag <- min(1, b_diag (1/2 / f)^(1/N)), f the fraction of chains whose
// configuration has s = s' on every site (f = 0 counts as 1/4).
__global__ void __launch_bounds__(NT) k_update_b(Prob P, int n, const uint8_t* configs, double* b_diag) {
  __shared__ double red[NT];
  double cnt = 0.0;
  for (int ch = threadIdx.x; ch < n; ch += NT) {
    const uint8_t* S = configs + (size_t)ch * P.N;
    bool diag = true;
    for (int i = 0; i < P.N; ++i) diag = diag && (ket_of(P, S[i]) == bra_of(P, S[i]));
    cnt += diag ? 1.0 : 0.0;
  }
  cnt = wg_sum(cnt, red);
  if (threadIdx.x == 0) {
    double f = cnt / (double)n;
    if (f == 0.0) f = 0.25;
    const double b = b_diag[0] * pow(0.5 / f, 1.0 / (double)P.N);
    b_diag[0] = b < 1.0 ? b : 1.0;
  }
}

// w_i = exp(2 log|rho_i| - log p_i - max_j (...)), 0 where either is -inf.
__global__ void __launch_bounds__(1024) k_importance_weights(int64_t n, const double* log_abs, const double* log_p,
                                                              double* w) {
  __shared__ double red[1024];
  const int tid = threadIdx.x;
  double m = -INFINITY;
  for (int64_t i = tid; i < n; i += 1024) {
    const double v = 2.0 * log_abs[i] - log_p[i];
    if (log_abs[i] > -INFINITY && log_p[i] > -INFINITY && v > m) m = v;
  }
  red[tid] = m;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  m = red[0];
  for (int64_t i = tid; i < n; i += 1024) {
    const bool ok = log_abs[i] > -INFINITY && log_p[i] > -INFINITY;
    w[i] = ok ? exp(2.0 * log_abs[i] - log_p[i] - m) : 0.0;
  }
}

}  // namespace

DirectLayout direct_layout(const Prob& P, const Prob& Q) {
  // sizes from the actual bond dimensions of every site of every row (the
  // compressed tops of P, the compressed double-layer bottoms of Q)
  Geo g, gq;
  build_geo(P, g);
  build_geo(Q, gq);
  int64_t tds = 1, env = 1, x0 = 1, x1 = 1, bs2 = 1;
  auto mx = [](int64_t& m, int64_t v) { m = v > m ? v : m; };
  for (int r = 0; r < P.L1; ++r)
    for (int c = 0; c < P.L2; ++c) {
      const int64_t ta = r ? (int64_t)g.ba[0][r - 1][c] * g.ba[0][r - 1][c] : 1;
      const int64_t tb = r ? (int64_t)g.bb[0][r - 1][c] * g.bb[0][r - 1][c] : 1;
      int Dl, Du, Dr, Dd;
      leg_dims(P, r, c, Dl, Du, Dr, Dd);
      const int64_t nl = Dl * Dl, nu = Du * Du, nr = Dr * Dr, nd = Dd * Dd;
      const bool below = r + 1 <= P.L1 - 1;
      const int64_t qa = below ? gq.ba[1][r + 1][c] : 1, qb = below ? gq.bb[1][r + 1][c] : 1;
      mx(tds, ta * nu * tb);
      mx(env, ta * nl * qa);           // L_c and R_c
      mx(env, tb * nr * qb);           // L_{c+1} and R_{c+1}
      mx(x0, qa * nd * tb * nr);       // right step, first stage
      mx(x1, nl * nu * qa * tb);       // right step, second stage
      mx(x0, nl * qa * nu * tb);       // left step and site environment, first stage
      mx(x1, qa * tb * nr * nd);       // left step, second stage
      mx(x1, nl * nu * tb * nd * qb);  // site environment, second stage
      mx(bs2, nl * nu * nr * nd);
    }
  auto pad = [](int64_t x) { return (x + 31) & ~(int64_t)31; };
  DirectLayout L;
  L.TDS = pad(tds);
  L.ENV = pad(env);
  int64_t off = 0;
  L.off_td = off;  off += (int64_t)P.L2 * L.TDS;
  L.off_R = off;   off += (int64_t)(P.L2 + 1) * L.ENV;
  L.off_L = off;   off += 2 * L.ENV;
  L.off_X0 = off;  off += pad(x0);
  L.off_X1 = off;  off += pad(x1);
  L.off_env = off; off += pad(bs2);
  L.off_Px = off;  off += pad(bs2);
  L.stride = off;
  L.x1 = x0 > x1 ? x0 : x1;
  if (bs2 > L.x1) L.x1 = bs2;
  return L;
}

hipError_t launch_double_layer(const Prob& P, const Prob& Q, const double* theta, double* eth, uint8_t* cfg_q,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_double_layer, dim3(P.N), dim3(NT), 0, st, P, Q, theta, eth, cfg_q);
  return hipGetLastError();
}

hipError_t launch_direct_row(const Prob& P, const Prob& Q, const DirectLayout& L, int n, int r, const double* theta,
                             const double* eth, uint8_t* configs, double* ws, const double* wsq, double* dws,
                             uint64_t seed, uint64_t draw, int reweight, const double* b_diag, double* log_p,
                             int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_direct_row, dim3(n), dim3(NT), 0, st, P, Q, L, theta, eth, configs, ws, wsq, dws, r, seed,
                     draw, reweight, b_diag, log_p, status);
  return hipGetLastError();
}

hipError_t launch_update_b(const Prob& P, int n, const uint8_t* configs, double* b_diag, hipStream_t st) {
  hipLaunchKernelGGL(k_update_b, dim3(1), dim3(NT), 0, st, P, n, configs, b_diag);
  return hipGetLastError();
}

hipError_t launch_importance_weights(int64_t n, const double* log_abs, const double* log_p, double* w,
                                     hipStream_t st) {
  hipLaunchKernelGGL(k_importance_weights, dim3(1), dim3(1024), 0, st, n, log_abs, log_p, w);
  return hipGetLastError();
}

}  // namespace peps
