// LDS-resident boundary-row compression (the general-shape fallback, one
// workgroup per chain, FP64), the per-sample output kernel and the local
// values of the diagonal observables.
#include <math.h>

#include "peps_chain.hpp"
#include "peps_common.hpp"
#include "peps_kernels.hpp"
#include "peps_linalg.hpp"

namespace peps {

// Mixed precision: bars of the error estimates above which a sample is
// measured again with the FP64 strips (k_redo_flags): the relative error of
// a one-row strip amplitude (O rows and log|psi| follow it: the O error
// relative to the row's largest entry stayed below 2.1 times the estimate),
// and the local-energy error against the scale of the precision bar (the
// estimate never fell below 1.37 times the true error).  Set from measured
// FP32 errors of the 8x8, D = 4, chi = 16 workload (two random states and a
// cooled one, 3 x 1024 samples), for a worst remaining error near a third of
// the mixed bar of 1e-4.
#ifndef PEPS_AMP_TOL
#define PEPS_AMP_TOL 3.0e-5
#endif
constexpr double AMP_TOL = PEPS_AMP_TOL;
constexpr double E_TOL = 5.0e-5;

// ---------------------------------------------------------------------------
// Compression of one boundary row: top[r] = C(top[r-1] o M_r) (dir 0) or
// bot[r] = C(M_r o bot[r+1]) (dir 1), for every chain.
__global__ void __launch_bounds__(NT) k_compress(Prob P, int dir, int r, const double* __restrict__ theta,
                                                 const uint8_t* __restrict__ configs, double* ws,
                                                 int32_t* status) {
  extern __shared__ double dyn[];
  __shared__ Geo geo;
  __shared__ double red[NT];
  __shared__ double tau[256];
  __shared__ double sig[256];
  __shared__ int rnk[256];
  __shared__ int flags[2];
  __shared__ int sa[MAX_L], sp[MAX_L], sb[MAX_L];
  __shared__ double one;
  const int tid = threadIdx.x;
  const int ch = blockIdx.x;
  if (tid == 0) {
    build_geo(P, geo);
    one = 1.0;
  }
  __syncthreads();
  ChainWS w = chain_ws(P, ws, ch);
  const uint8_t* cfg = configs + (size_t)ch * P.N;
  double* bnd = dir == 0 ? w.top : w.bot;
  double* lsb = dir == 0 ? w.lstop : w.lsbot;
  double* outT = bnd + (size_t)r * P.L2 * P.TS;
  const bool has_prev = dir == 0 ? (r > 0) : (r < P.L1 - 1);
  const int rp = dir == 0 ? r - 1 : r + 1;
  const double ls_prev = has_prev ? lsb[rp] : 0.0;

  // 1. absorb the row into the boundary: B_c[(a,l)][p][(b,r)]
  for (int c = 0; c < P.L2; ++c) {
    int Dl, Du, Dr, Dd;
    leg_dims(P, r, c, Dl, Du, Dr, Dd);
    const int i = r * P.L2 + c;
    const double* W = theta + geo.poff[i] + (size_t)digit_at(P, cfg, i) * (Dl * Du * Dr * Dd);
    const double* A;
    int a, q, b;
    if (has_prev) {
      A = bnd + ((size_t)rp * P.L2 + c) * P.TS;
      a = geo.ba[dir][rp][c];
      b = geo.bb[dir][rp][c];
      q = dir == 0 ? Du : Dd;
    } else {
      A = &one;
      a = b = q = 1;
    }
    const int pp = dir == 0 ? Dd : Du;
    double* Bc = w.B + (size_t)c * P.BS;
    const int total = a * Dl * pp * b * Dr;
    for (int idx = tid; idx < total; idx += NT) {
      int rr = idx % Dr, t = idx / Dr;
      int bq = t % b; t /= b;
      int p = t % pp; t /= pp;
      int l = t % Dl, aa = t / Dl;
      double s = 0.0;
      for (int x = 0; x < q; ++x) {
        double Av = A[(aa * q + x) * b + bq];
        double Wv = dir == 0 ? W[((l * Du + x) * Dr + rr) * Dd + p] : W[((l * Du + p) * Dr + rr) * Dd + x];
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

  // 2. left-to-right thin QR; X (LDS) carries R_{c-1} B_c between steps
  double* X = dyn;
  for (int c = 0; c < P.L2 - 1; ++c) {
    const int m = sa[c] * sp[c], n = sb[c];
    double* Bc = w.B + (size_t)c * P.BS;
    if (c == 0) {
      for (int idx = tid; idx < m * n; idx += NT) X[idx] = Bc[idx];
      __syncthreads();
    }
    wg_householder(X, m, n, n, tau, red);
    const int k = m < n ? m : n;
    for (int idx = tid; idx < k * n; idx += NT) {
      int i = idx / n, j = idx % n;
      w.tmp[idx] = j >= i ? X[i * n + j] : 0.0;
    }
    __syncthreads();
    wg_form_q(X, m, n, n, tau, red);
    for (int idx = tid; idx < m * k; idx += NT) {
      int i = idx / k, j = idx % k;
      Bc[idx] = X[i * n + j];
    }
    __syncthreads();
    const int rest = sp[c + 1] * sb[c + 1];
    const double* Bn = w.B + (size_t)(c + 1) * P.BS;
    for (int idx = tid; idx < k * rest; idx += NT) {
      int i = idx / rest, q = idx % rest;
      double s = 0.0;
      for (int j = i; j < n; ++j) s += w.tmp[i * n + j] * Bn[(size_t)j * rest + q];
      X[idx] = s;
    }
    __syncthreads();
    if (tid == 0) {
      sb[c] = k;
      sa[c + 1] = k;
    }
    __syncthreads();
  }
  {
    const int c = P.L2 - 1;
    const int tot = sa[c] * sp[c] * sb[c];
    double* Bc = w.B + (size_t)c * P.BS;
    for (int idx = tid; idx < tot; idx += NT) Bc[idx] = X[idx];
    __syncthreads();
  }

  // 3. right-to-left SVD truncation to chi
  for (int c = P.L2 - 1; c >= 1; --c) {
    const int a = sa[c], nb = sp[c] * sb[c];
    const bool tr = a < nb;
    const int mg = tr ? nb : a, ng = tr ? a : nb;
    const int cs = mg | 1;
    double* G = dyn;
    double* V = dyn + (size_t)cs * ng;
    const double* M = w.B + (size_t)c * P.BS;
    for (int idx = tid; idx < mg * ng; idx += NT) {
      int j = idx / mg, i = idx % mg;
      G[j * cs + i] = tr ? M[j * nb + i] : M[i * nb + j];
    }
    for (int idx = tid; idx < ng * ng; idx += NT) {
      int j = idx / ng, i = idx % ng;
      V[idx] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    wg_jacobi(G, mg, ng, cs, V, ng, flags);
    for (int j = tid; j < ng; j += NT) {
      double s = 0.0;
      for (int i = 0; i < mg; ++i) s += G[j * cs + i] * G[j * cs + i];
      sig[j] = rank_norm(s, status);
    }
    __syncthreads();
    for (int j = tid; j < ng; j += NT) {
      int rk = 0;
      for (int q = 0; q < ng; ++q)
        if (sig[q] > sig[j] || (sig[q] == sig[j] && q < j)) ++rk;
      rnk[j] = rk;
    }
    __syncthreads();
    const int k2 = P.chi < ng ? P.chi : ng;
    double* Vt = outT + (size_t)c * P.TS;
    for (int idx = tid; idx < a * ng; idx += NT) {
      int i = idx / ng, j = idx % ng;
      int q = rnk[j];
      if (q < k2) w.tmp[i * k2 + q] = tr ? V[j * ng + i] * sig[j] : G[j * cs + i];
    }
    for (int idx = tid; idx < nb * ng; idx += NT) {
      int e = idx / ng, j = idx % ng;
      int q = rnk[j];
      if (q < k2) Vt[q * nb + e] = tr ? (sig[j] > 0.0 ? G[j * cs + e] / sig[j] : 0.0) : V[j * ng + e];
    }
    __syncthreads();
    const int m2 = sa[c - 1] * sp[c - 1];
    double* Bp = w.B + (size_t)(c - 1) * P.BS;
    double* Y = dyn;
    for (int idx = tid; idx < m2 * k2; idx += NT) {
      int i = idx / k2, q = idx % k2;
      double s = 0.0;
      for (int j = 0; j < a; ++j) s += Bp[(size_t)i * a + j] * w.tmp[j * k2 + q];
      Y[idx] = s;
    }
    __syncthreads();
    for (int idx = tid; idx < m2 * k2; idx += NT) Bp[idx] = Y[idx];
    if (tid == 0) {
      sb[c - 1] = k2;
      sa[c] = k2;
    }
    __syncthreads();
  }

  // 4. normalise site 0 and accumulate the log-scale
  const int tot0 = sa[0] * sp[0] * sb[0];
  double part = 0.0;
  for (int idx = tid; idx < tot0; idx += NT) part += w.B[idx] * w.B[idx];
  const double nrm = sqrt(wg_sum(part, red));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int idx = tid; idx < tot0; idx += NT) outT[idx] = w.B[idx] * inv;
  if (tid == 0) {
    lsb[r] = nrm > 0.0 ? ls_prev + log(nrm) : -INFINITY;
    for (int c = 0; c < P.L2; ++c)
      if (sa[c] != geo.ba[dir][r][c] || sb[c] != geo.bb[dir][r][c]) set_status(status, PEPS_ERR_UNSUPPORTED);
  }
  // 5. FP32 copy of the row for the mixed-precision strips
  if (P.mixed) {
    __syncthreads();
    float* o32 = (float*)(ws + (size_t)ch * P.chain_stride + (dir == 0 ? P.off_top32 : P.off_bot32)) +
                 (size_t)r * P.L2 * P.TS;
    for (int idx = tid; idx < P.L2 * P.TS; idx += NT) o32[idx] = (float)outT[idx];
  }
}

// Local values (A(s) + A(s')) / 2 of M_z, M_z^2, particle number and double
// occupancy for each sample; every term is a multiple of 1/8, so the sums
// are exact.
__global__ void k_observables(Prob P, int64_t n, const uint8_t* __restrict__ configs, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint8_t* S = configs + k * P.N;
  double acc[PEPS_N_OBS] = {0.0, 0.0, 0.0, 0.0};
  for (int side = 0; side < 2; ++side) {
    double mz = 0.0, np_ = 0.0, dc = 0.0;
    for (int i = 0; i < P.N; ++i) {
      const int s = side == 0 ? S[i] / P.d : S[i] % P.d;
      if (P.model == PEPS_MODEL_HEISENBERG) {
        mz += 0.5 - s;
      } else {
        const int nu = s & 1, nd = (s >> 1) & 1;
        mz += 0.5 * (nu - nd);
        np_ += nu + nd;
        dc += nu * nd;
      }
    }
    acc[0] += 0.5 * mz;
    acc[1] += 0.5 * mz * mz;
    acc[2] += 0.5 * np_;
    acc[3] += 0.5 * dc;
  }
#pragma unroll
  for (int q = 0; q < PEPS_N_OBS; ++q) out[k * PEPS_N_OBS + q] = acc[q];
}

hipError_t launch_observables(const Prob& P, int64_t n, const uint8_t* configs, double* out, hipStream_t st) {
  const int bs = 128;
  hipLaunchKernelGGL(k_observables, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st, P, n, configs, out);
  return hipGetLastError();
}

// Diagonal energy, sum of the parts, and the per-sample outputs.
// Mixed precision: the first pass (redo = 0) also records the sample's local
// energy and its error estimate from the FP32 strips, from which k_redo_flags
// decides whether the sample is measured again in FP64; the second pass
// (redo = 1) rewrites the outputs of the flagged samples from their FP64
// parts.
__global__ void k_finalize(Prob P, int n, const uint8_t* configs, double* ws, double* log_abs, int8_t* sign,
                           double* e_loc, int64_t out_off, int want_e, int redo, int32_t* status) {
  const int ch = blockIdx.x * blockDim.x + threadIdx.x;
  if (ch >= n) return;
  double* ep = ws + (size_t)ch * P.chain_stride + P.off_epart;
  if (redo && ep[epart_flag(P)] == 0.0) return;
  const uint8_t* S = configs + (size_t)ch * P.N;
  const double la = ep[2 * P.L1];
  // log|psi| and the sign come from the last row's strip: rewritten when that
  // strip was measured again for its amplitude (never for the energy alone,
  // so that they do not depend on whether the energy was asked for)
  const bool write_amp = !redo || ((((uint32_t)ep[epart_mask(P)]) >> (P.L1 - 1)) & 1u);
  if (write_amp) {
    if (log_abs) log_abs[out_off + ch] = la;
    if (sign) sign[out_off + ch] = (int8_t)ep[2 * P.L1 + 1];
    if (isnan(la) || la == INFINITY) set_status(status, PEPS_ERR_NONFINITE);   // -inf: a zero amplitude
  }
  if (!want_e || !e_loc) return;
  double diag = 0.0;
  if (P.model == PEPS_MODEL_HEISENBERG) {
    for (int side = 0; side < 2; ++side) {
      for (int rr = 0; rr < P.L1; ++rr)
        for (int c = 0; c < P.L2; ++c) {
          const int i = rr * P.L2 + c;
          const int zi = 1 - 2 * (side == 0 ? S[i] / P.d : S[i] % P.d);
          if (c + 1 < P.L2) {
            const int zj = 1 - 2 * (side == 0 ? S[i + 1] / P.d : S[i + 1] % P.d);
            diag += P.J1 * 0.25 * zi * zj;
          }
          if (rr + 1 < P.L1) {
            const int zj = 1 - 2 * (side == 0 ? S[i + P.L2] / P.d : S[i + P.L2] % P.d);
            diag += P.J1 * 0.25 * zi * zj;
          }
          if (P.J2 != 0.0 && rr + 1 < P.L1) {
            if (c + 1 < P.L2) {
              const int zj = 1 - 2 * (side == 0 ? S[i + P.L2 + 1] / P.d : S[i + P.L2 + 1] % P.d);
              diag += P.J2 * 0.25 * zi * zj;
            }
            if (c >= 1) {
              const int zj = 1 - 2 * (side == 0 ? S[i + P.L2 - 1] / P.d : S[i + P.L2 - 1] % P.d);
              diag += P.J2 * 0.25 * zi * zj;
            }
          }
        }
    }
  }
  if (P.model == PEPS_MODEL_HUBBARD) {
    // U n_up n_dn - mu (n_up + n_dn) on every site, ket and bra digits;
    // J2 S^z_i S^z_j on next-nearest-neighbour pairs, S^z = (n_up - n_dn)/2
    for (int side = 0; side < 2; ++side)
      for (int i = 0; i < P.N; ++i) {
        const int dg = side == 0 ? S[i] / P.d : S[i] % P.d;
        const int nu = dg & 1, nd = (dg >> 1) & 1;
        diag += P.U * (nu * nd) - P.mu * (nu + nd);
        const int rr = i / P.L2, c = i % P.L2;
        if (P.J2 != 0.0 && rr + 1 < P.L1) {
          const int zi = nu - nd;   // 2 S^z_i
          for (int dc = -1; dc <= 1; dc += 2) {
            if (c + dc < 0 || c + dc >= P.L2) continue;
            const int dj = side == 0 ? S[i + P.L2 + dc] / P.d : S[i + P.L2 + dc] % P.d;
            const int zj = (dj & 1) - ((dj >> 1) & 1);
            diag += P.J2 * 0.25 * zi * zj;
          }
        }
      }
  }
  double e = diag;
  for (int q = 0; q < 2 * P.L1 - 1; ++q) e += ep[q];
  e_loc[out_off + ch] = e;
  if (P.mixed && !redo) ep[epart_e32(P)] = e;
  if (!isfinite(e)) set_status(status, PEPS_ERR_NONFINITE);
}

// Mixed precision: which row strips of which samples are measured again in
// FP64.  Per strip, e = max(dev, kap) estimates the relative rounding error
// of its amplitude (see the FP32 strip kernels).  Every one-row strip with
// e > AMP_TOL is measured again with its O rows (its amplitude sets those
// rows, its in-row energy terms and, for the last row, log|psi|).  With the
// local energy wanted, the sample's energy error is then estimated as the
// sum over the strips not yet listed of max(e, u32) a (a: the summed
// magnitudes of the strip's terms), and while it exceeds E_TOL max(|E_loc|,
// mean |E_loc|) (the scale of the precision bar, the mean over the batch's
// finite local energies) the strip of largest contribution is listed too
// (energy only).  Items are listed per chain in increasing chain order, as
// chain * 64 + kind (kind r < L1: one-row strip r; L1 + r: two-row strip
// r): list[0] = count, then the items.  One workgroup, fixed order; thread
// t owns a contiguous block of chains.
__global__ void __launch_bounds__(NT) k_redo_flags(Prob P, int n, double* ws, int want_e, int32_t* list) {
  __shared__ double red[NT];
  __shared__ int cnt[NT];
  const int tid = threadIdx.x;
  const int per = (n + NT - 1) / NT;
  const int c0 = tid * per < n ? tid * per : n;
  const int c1 = c0 + per < n ? c0 + per : n;
  double s = 0.0, c = 0.0;
  if (want_e)
    for (int ch = c0; ch < c1; ++ch) {
      const double e = ws[(size_t)ch * P.chain_stride + P.off_epart + epart_e32(P)];
      if (isfinite(e)) {
        s += fabs(e);
        c += 1.0;
      }
    }
  s = wg_sum(s, red);
  c = wg_sum(c, red);
  const double mean_abs = c > 0.0 ? s / c : 0.0;
  const double u32 = 0x1.0p-24;
  int mine = 0;
  for (int ch = c0; ch < c1; ++ch) {
    double* ep = ws + (size_t)ch * P.chain_stride + P.off_epart;
    uint32_t m_amp = 0, m1 = 0, m2 = 0;
    double err = 0.0;
    bool bad = false;
    for (int r = 0; r < P.L1; ++r) {
      const double* q = ep + epart_err1(P) + 3 * r;
      const double e = fmax(q[0], q[1]);
      if (!(e <= AMP_TOL)) m_amp |= 1u << r;   // NaN included
      err += fmax(e, u32) * q[2];
      bad = bad || isnan(e) || isnan(q[2]);
    }
    for (int r = 0; r + 1 < P.L1; ++r) {
      const double* q = ep + epart_err2(P) + 3 * r;
      err += fmax(fmax(q[0], q[1]), u32) * q[2];
      bad = bad || isnan(q[0]) || isnan(q[1]) || isnan(q[2]);
    }
    if (bad) err = NAN;
    ep[epart_e32(P) + 1] = err;
    m1 = m_amp;
    if (want_e) {
      const double bar = E_TOL * fmax(fabs(ep[epart_e32(P)]), mean_abs);
      if (bad) {
        m1 = (P.L1 >= 32) ? 0xffffffffu : ((1u << P.L1) - 1u);
        m2 = (P.L1 - 1 >= 32) ? 0xffffffffu : ((1u << (P.L1 - 1)) - 1u);
      } else {
        // the remaining estimate, then the largest remaining contributions
        double rem = 0.0;
        for (int r = 0; r < P.L1; ++r) {
          const double* q = ep + epart_err1(P) + 3 * r;
          if (!((m1 >> r) & 1u)) rem += fmax(fmax(q[0], q[1]), u32) * q[2];
        }
        for (int r = 0; r + 1 < P.L1; ++r) {
          const double* q = ep + epart_err2(P) + 3 * r;
          rem += fmax(fmax(q[0], q[1]), u32) * q[2];
        }
        while (!(rem <= bar)) {
          double best = -1.0;
          int bk = -1;
          for (int r = 0; r < P.L1; ++r) {
            if ((m1 >> r) & 1u) continue;
            const double* q = ep + epart_err1(P) + 3 * r;
            const double v = fmax(fmax(q[0], q[1]), u32) * q[2];
            if (v > best) { best = v; bk = r; }
          }
          for (int r = 0; r + 1 < P.L1; ++r) {
            if ((m2 >> r) & 1u) continue;
            const double* q = ep + epart_err2(P) + 3 * r;
            const double v = fmax(fmax(q[0], q[1]), u32) * q[2];
            if (v > best) { best = v; bk = P.L1 + r; }
          }
          if (bk < 0) break;
          if (bk < P.L1) m1 |= 1u << bk;
          else m2 |= 1u << (bk - P.L1);
          rem -= best;
        }
      }
    }
    ep[epart_mask(P)] = (double)m_amp;
    ep[epart_mask(P) + 1] = (double)m1;
    ep[epart_mask(P) + 2] = (double)m2;
    ep[epart_flag(P)] = m_amp ? 2.0 : ((m1 | m2) ? 1.0 : 0.0);
    mine += __popc(m1) + __popc(m2);
  }
  // inclusive scan of the per-thread item counts, then each thread lists its own
  cnt[tid] = mine;
  __syncthreads();
  for (int off = 1; off < NT; off <<= 1) {
    const int v = tid >= off ? cnt[tid - off] : 0;
    __syncthreads();
    cnt[tid] += v;
    __syncthreads();
  }
  int pos = cnt[tid] - mine;
  for (int ch = c0; ch < c1; ++ch) {
    const double* ep = ws + (size_t)ch * P.chain_stride + P.off_epart;
    const uint32_t m1 = (uint32_t)ep[epart_mask(P) + 1], m2 = (uint32_t)ep[epart_mask(P) + 2];
    for (int r = 0; r < P.L1; ++r)
      if ((m1 >> r) & 1u) list[1 + pos++] = ch * 64 + r;
    for (int r = 0; r + 1 < P.L1; ++r)
      if ((m2 >> r) & 1u) list[1 + pos++] = ch * 64 + P.L1 + r;
  }
  if (tid == NT - 1) list[0] = cnt[NT - 1];
}

hipError_t launch_redo_flags(const Prob& P, int n, double* ws, int want_e, int32_t* list, hipStream_t st) {
  hipLaunchKernelGGL(k_redo_flags, dim3(1), dim3(NT), 0, st, P, n, ws, want_e, list);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host-side launchers.

static size_t compress_lds_bytes(const Prob& P) {
  const size_t cd = (size_t)P.chi * P.D;
  size_t qr = cd * P.D * cd;
  size_t svd = cd * cd + ((cd | 1) + 1) * cd + cd * cd;
  return (qr > svd ? qr : svd) * sizeof(double);
}

size_t compress_dyn_lds(const Prob& P) { return compress_lds_bytes(P); }

bool compress_in_lds(const Prob& P) { return compress_lds_bytes(P) <= COMPRESS_DYN_LDS_MAX; }

hipError_t launch_compress(const Prob& P, int n, int dir, int r, const double* theta, const uint8_t* configs,
                           double* ws, int32_t* status, hipStream_t st) {
  const size_t lds = compress_lds_bytes(P);
  // beyond the default 64 KB of dynamic LDS the kernel's limit is raised on
  // the current device, at every such launch (no state kept between calls)
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_compress, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)COMPRESS_DYN_LDS_MAX);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_compress, dim3(n), dim3(NT), lds, st, P, dir, r, theta, configs, ws, status);
  return hipGetLastError();
}

hipError_t launch_finalize(const Prob& P, int n, const uint8_t* configs, double* ws, double* log_abs, int8_t* sign,
                           double* e_loc, int64_t out_off, int want_e, int redo, int32_t* status, hipStream_t st) {
  const int bs = 128;
  hipLaunchKernelGGL(k_finalize, dim3((n + bs - 1) / bs), dim3(bs), 0, st, P, n, configs, ws, log_abs, sign, e_loc,
                     out_off, want_e, redo, status);
  return hipGetLastError();
}

// Range check of the configuration digits of a call: any digit >= d^2
// records PEPS_ERR_ARG (the kernels read such a digit as 0).
__global__ void k_check_digits(int64_t nbytes, int d2, const uint8_t* __restrict__ configs, int32_t* status) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nbytes; i += (int64_t)gridDim.x * blockDim.x)
    bad |= configs[i] >= d2;
  if (bad) set_status(status, PEPS_ERR_ARG);
}

hipError_t launch_check_digits(const Prob& P, int64_t n, const uint8_t* configs, int32_t* status, hipStream_t st) {
  const int64_t nbytes = n * P.N;
  if (nbytes <= 0) return hipSuccess;
  int64_t blocks = (nbytes + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_check_digits, dim3((unsigned)blocks), dim3(256), 0, st, nbytes, P.d2, configs, status);
  return hipGetLastError();
}

// Weighted means and per-chain standard errors of k per-sample quantities
// (one workgroup per quantity, fixed summation order).  Weights: explicit,
// else |rho|^(2 - alpha) relative to the largest amplitude from log_abs,
// else uniform.
__global__ void __launch_bounds__(NT) k_sample_stats(Prob P, int n_sweeps, int n_chains, int k,
                                                     const double* __restrict__ values,
                                                     const double* __restrict__ weights,
                                                     const double* __restrict__ log_abs, double* out) {
  __shared__ double red[NT];
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t n_s = (int64_t)n_sweeps * n_chains;
  const bool wgt = weights == nullptr && log_abs != nullptr && P.alpha != 2;
  double lmax = -INFINITY;
  if (wgt) {
    for (int64_t i = tid; i < n_s; i += NT) lmax = fmax(lmax, log_abs[i]);
    red[tid] = lmax;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
      __syncthreads();
    }
    lmax = red[0];
    __syncthreads();
  }
  auto weight = [&](int64_t i) {
    return weights ? weights[i] : (wgt ? exp((double)(2 - P.alpha) * (log_abs[i] - lmax)) : 1.0);
  };
  double sw = 0.0, sv = 0.0;
  for (int64_t i = tid; i < n_s; i += NT) {
    const double wi = weight(i);
    sw += wi;
    sv += wi * values[i * k + q];
  }
  sw = wg_sum(sw, red);
  sv = wg_sum(sv, red);
  const double mean = sv / sw;
  // per-chain weighted means (thread-strided over chains), their mean and
  // sample variance
  double s1 = 0.0, s2 = 0.0;
  for (int c = tid; c < n_chains; c += NT) {
    double cw = 0.0, cv = 0.0;
    for (int t = 0; t < n_sweeps; ++t) {
      const int64_t i = (int64_t)t * n_chains + c;
      const double wi = weight(i);
      cw += wi;
      cv += wi * values[i * k + q];
    }
    const double m = cv / cw;
    s1 += m;
    s2 += m * m;
  }
  s1 = wg_sum(s1, red);
  s2 = wg_sum(s2, red);
  if (tid == 0) {
    out[2 * q] = mean;
    double se = 0.0;
    if (n_chains > 1) {
      const double mc = s1 / n_chains;
      const double var = fmax(s2 - n_chains * mc * mc, 0.0) / (n_chains - 1);
      se = sqrt(var / n_chains);
    }
    out[2 * q + 1] = se;
  }
}

hipError_t launch_sample_stats(const Prob& P, int n_sweeps, int n_chains, int k, const double* values,
                               const double* weights, const double* log_abs, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sample_stats, dim3(k), dim3(NT), 0, st, P, n_sweeps, n_chains, k, values, weights, log_abs,
                     out);
  return hipGetLastError();
}

}  // namespace peps
