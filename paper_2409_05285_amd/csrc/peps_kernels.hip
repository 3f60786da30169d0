// Per-chain kernels of the sampling / evaluation path (one workgroup per
// chain, FP64): boundary-MPS compression, Metropolis passes over one row
// (one-row strip) and over a pair of rows (two-row strip), and the
// measurement of E_loc, O rows and log|psi|.
#include <math.h>

#include "peps_common.hpp"
#include "peps_contract.hpp"
#include "peps_kernels.hpp"
#include "peps_linalg.hpp"

namespace peps {

struct ChainWS {
  double *top, *lstop, *bot, *lsbot, *B, *tmp, *R, *L, *X, *epart;
};

__device__ inline ChainWS chain_ws(const Prob& P, double* ws, int ch) {
  double* base = ws + (size_t)ch * P.chain_stride;
  ChainWS w;
  w.top = base + P.off_top;
  w.lstop = base + P.off_lstop;
  w.bot = base + P.off_bot;
  w.lsbot = base + P.off_lsbot;
  w.B = base + P.off_B;
  w.tmp = base + P.off_tmp;
  w.R = base + P.off_R;
  w.L = base + P.off_L;
  w.X = base + P.off_X;
  w.epart = base + P.off_epart;
  return w;
}

// Boundary tensors and dimensions of the strip around row r (one-row:
// top[r-1] and bot[r+1]; two-row: top[r-1] and bot[r+2]), with the
// trivial boundary (one element equal to 1) outside the lattice.
struct StripCtx {
  const double* T[MAX_L];
  const double* B[MAX_L];
  Dim3 tD[MAX_L];
  Dim3 bD[MAX_L];
};

__device__ inline void build_strip(const Prob& P, const Geo& g, const ChainWS& w, int r, int rb,
                                   const double* one, StripCtx& s) {
  if (threadIdx.x != 0) return;
  for (int c = 0; c < P.L2; ++c) {
    int Dl, Du, Dr, Dd;
    leg_dims(P, r, c, Dl, Du, Dr, Dd);
    if (r >= 1) {
      s.T[c] = w.top + ((size_t)(r - 1) * P.L2 + c) * P.TS;
      s.tD[c] = Dim3{g.ba[0][r - 1][c], Du, g.bb[0][r - 1][c]};
    } else {
      s.T[c] = one;
      s.tD[c] = Dim3{1, 1, 1};
    }
    if (rb <= P.L1 - 1) {
      int Dl2, Du2, Dr2, Dd2;
      leg_dims(P, rb, c, Dl2, Du2, Dr2, Dd2);
      s.B[c] = w.bot + ((size_t)rb * P.L2 + c) * P.TS;
      s.bD[c] = Dim3{g.ba[1][rb][c], Du2, g.bb[1][rb][c]};
    } else {
      s.B[c] = one;
      s.bD[c] = Dim3{1, 1, 1};
    }
  }
}

__device__ inline const double* slice_ptr(const Prob& P, const Geo& g, const double* theta, int r, int c, int S) {
  return theta + g.poff[r * P.L2 + c] + (size_t)S * block_size(P, r, c);
}

__device__ inline Dim4 wdim(const Prob& P, int r, int c) {
  int Dl, Du, Dr, Dd;
  leg_dims(P, r, c, Dl, Du, Dr, Dd);
  return Dim4{Dl, Du, Dr, Dd};
}

__device__ inline int slot_base(const Prob& P, int r) {
  return r * (P.nb_moves * (P.L2 - 1) + P.ns_moves * P.L2 + P.nb_moves * P.L2);
}

// Proposals (shared by the sweep and the local energy).  Digit helpers.
__device__ inline int ket_of(const Prob& P, int S) { return S / P.d; }
__device__ inline int bra_of(const Prob& P, int S) { return S % P.d; }
__device__ inline int merge(const Prob& P, int s, int sp) { return s * P.d + sp; }

// Exchange proposal k on a bond (sites with states Sa, Sb).  Returns false
// when it would not change the configuration.
__device__ inline bool bond_proposal(const Prob& P, int Sa, int Sb, int k, int& na, int& nb) {
  if (P.model == PEPS_MODEL_HEISENBERG) {
    if (k == 0) {
      int a = ket_of(P, Sa), b = ket_of(P, Sb);
      if (a == b) return false;
      na = merge(P, b, bra_of(P, Sa));
      nb = merge(P, a, bra_of(P, Sb));
    } else {
      int a = bra_of(P, Sa), b = bra_of(P, Sb);
      if (a == b) return false;
      na = merge(P, ket_of(P, Sa), b);
      nb = merge(P, ket_of(P, Sb), a);
    }
    return true;
  }
  int side = k / 2, sg = k % 2;
  int da = side == 0 ? ket_of(P, Sa) : bra_of(P, Sa);
  int db = side == 0 ? ket_of(P, Sb) : bra_of(P, Sb);
  if (((da >> sg) & 1) == ((db >> sg) & 1)) return false;
  int da2 = da ^ (1 << sg), db2 = db ^ (1 << sg);
  if (side == 0) {
    na = merge(P, da2, bra_of(P, Sa));
    nb = merge(P, db2, bra_of(P, Sb));
  } else {
    na = merge(P, ket_of(P, Sa), da2);
    nb = merge(P, ket_of(P, Sb), db2);
  }
  return true;
}

__device__ inline bool site_proposal(const Prob& P, int S, int k, int& ns) {
  int s = ket_of(P, S), sp = bra_of(P, S);
  if (P.model == PEPS_MODEL_HEISENBERG) {
    if (s != sp) return false;
    ns = merge(P, 1 - s, 1 - sp);
    return true;
  }
  if (((s >> k) & 1) != ((sp >> k) & 1)) return false;
  ns = merge(P, s ^ (1 << k), sp ^ (1 << k));
  return true;
}

__device__ inline bool metropolis(const Prob& P, double R, double u) {
  double wgt = P.alpha == 2 ? R * R : fabs(R);
  return u < fmin(1.0, wgt);
}

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
    const double* W = theta + geo.poff[i] + (size_t)cfg[i] * (Dl * Du * Dr * Dd);
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
      sig[j] = sqrt(s);
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
}

// ---------------------------------------------------------------------------
// Shared prologue of the strip kernels.
#define STRIP_PROLOGUE                                        \
  __shared__ Geo geo;                                         \
  __shared__ double red[NT];                                  \
  __shared__ StripCtx sc;                                     \
  __shared__ uint8_t S[MAX_SITES];                            \
  __shared__ double one;                                      \
  const int tid = threadIdx.x;                                \
  const int ch = blockIdx.x;                                  \
  ChainWS w = chain_ws(P, ws, ch);                            \
  uint8_t* cfg = (uint8_t*)configs + (size_t)ch * P.N;         \
  if (tid == 0) {                                             \
    build_geo(P, geo);                                        \
    one = 1.0;                                                \
  }                                                           \
  for (int i = tid; i < P.N; i += NT) S[i] = cfg[i];          \
  __syncthreads();

// One-row environments from the right: R_c (c = L2..0) at w.R + c*ES.
__device__ inline void right_envs1(const Prob& P, const Geo& g, const StripCtx& sc, const uint8_t* S,
                                   const double* theta, const ChainWS& w, int r) {
  if (threadIdx.x == 0) w.R[(size_t)P.L2 * P.ES] = 1.0;
  __syncthreads();
  for (int c = P.L2 - 1; c >= 0; --c) {
    const int i = r * P.L2 + c;
    rstep1(w.R + (size_t)c * P.ES, w.R + (size_t)(c + 1) * P.ES, sc.T[c], sc.tD[c],
           slice_ptr(P, g, theta, r, c, S[i]), wdim(P, r, c), sc.B[c], sc.bD[c], w.X, w.X + P.XS);
  }
}

__device__ inline void right_envs2(const Prob& P, const Geo& g, const StripCtx& sc, const uint8_t* S,
                                   const double* theta, const ChainWS& w, int r) {
  if (threadIdx.x == 0) w.R[(size_t)P.L2 * P.ES] = 1.0;
  __syncthreads();
  for (int c = P.L2 - 1; c >= 0; --c) {
    const int i = r * P.L2 + c, j = (r + 1) * P.L2 + c;
    rstep2(w.R + (size_t)c * P.ES, w.R + (size_t)(c + 1) * P.ES, sc.T[c], sc.tD[c],
           slice_ptr(P, g, theta, r, c, S[i]), wdim(P, r, c), slice_ptr(P, g, theta, r + 1, c, S[j]),
           wdim(P, r + 1, c), sc.B[c], sc.bD[c], w.X, w.X + P.XS);
  }
}

__device__ inline int env1_size(const Prob& P, const StripCtx& sc, int r, int c) {
  Dim4 wd = wdim(P, r, c);
  return sc.tD[c].n2 * wd.n2 * sc.bD[c].n2;
}

__device__ inline int env2_size(const Prob& P, const StripCtx& sc, int r, int c) {
  return sc.tD[c].n2 * wdim(P, r, c).n2 * wdim(P, r + 1, c).n2 * sc.bD[c].n2;
}

// Metropolis passes inside row r: horizontal exchanges, then site moves.
__global__ void __launch_bounds__(NT) k_moves1(Prob P, int r, const double* __restrict__ theta, uint8_t* configs,
                                               uint64_t seed, uint64_t gsweep, double* ws, int32_t* n_accept,
                                               int32_t* status) {
  STRIP_PROLOGUE
  build_strip(P, geo, w, r, r + 1, &one, sc);
  __syncthreads();
  int acc_h = 0, acc_s = 0;
  double* Lb[2] = {w.L, w.L + P.ES};
  double* tA = w.L + 2 * (size_t)P.ES;
  double* tB = w.L + 3 * (size_t)P.ES;
  double* X0 = w.X;
  double* X1 = w.X + P.XS;
  int slot = slot_base(P, r);

  // horizontal exchanges
  right_envs1(P, geo, sc, S, theta, w, r);
  double rho = w.R[0];
  const double* Lc = &one;
  int cur = 0;
  for (int c = 0; c < P.L2 - 1; ++c) {
    const int i = r * P.L2 + c, j = i + 1;
    for (int k = 0; k < P.nb_moves; ++k, ++slot) {
      int ni, nj;
      if (!bond_proposal(P, S[i], S[j], k, ni, nj)) continue;
      lstep1(tA, Lc, sc.T[c], sc.tD[c], slice_ptr(P, geo, theta, r, c, ni), wdim(P, r, c), sc.B[c], sc.bD[c], X0, X1);
      lstep1(tB, tA, sc.T[c + 1], sc.tD[c + 1], slice_ptr(P, geo, theta, r, c + 1, nj), wdim(P, r, c + 1),
             sc.B[c + 1], sc.bD[c + 1], X0, X1);
      const double rn = wg_dot(tB, w.R + (size_t)(c + 2) * P.ES, env1_size(P, sc, r, c + 1), red);
      bool acc = false;
      if (rho == 0.0) set_status(status, PEPS_ERR_ZERO_AMPLITUDE);
      else acc = metropolis(P, rn / rho, slot_uniform(seed, ch, gsweep, slot));
      if (acc) {
        if (tid == 0) { S[i] = (uint8_t)ni; S[j] = (uint8_t)nj; }
        rho = rn;
        ++acc_h;
      }
      __syncthreads();
    }
    lstep1(Lb[cur], Lc, sc.T[c], sc.tD[c], slice_ptr(P, geo, theta, r, c, S[i]), wdim(P, r, c), sc.B[c], sc.bD[c], X0, X1);
    Lc = Lb[cur];
    cur ^= 1;
  }

  // site moves
  right_envs1(P, geo, sc, S, theta, w, r);
  rho = w.R[0];
  Lc = &one;
  for (int c = 0; c < P.L2; ++c) {
    const int i = r * P.L2 + c;
    for (int k = 0; k < P.ns_moves; ++k, ++slot) {
      int ni;
      if (!site_proposal(P, S[i], k, ni)) continue;
      lstep1(tA, Lc, sc.T[c], sc.tD[c], slice_ptr(P, geo, theta, r, c, ni), wdim(P, r, c), sc.B[c], sc.bD[c], X0, X1);
      const double rn = wg_dot(tA, w.R + (size_t)(c + 1) * P.ES, env1_size(P, sc, r, c), red);
      bool acc = false;
      if (rho == 0.0) set_status(status, PEPS_ERR_ZERO_AMPLITUDE);
      else acc = metropolis(P, rn / rho, slot_uniform(seed, ch, gsweep, slot));
      if (acc) {
        if (tid == 0) S[i] = (uint8_t)ni;
        rho = rn;
        ++acc_s;
      }
      __syncthreads();
    }
    if (c < P.L2 - 1) {
      lstep1(Lb[cur], Lc, sc.T[c], sc.tD[c], slice_ptr(P, geo, theta, r, c, S[i]), wdim(P, r, c), sc.B[c], sc.bD[c], X0, X1);
      Lc = Lb[cur];
      cur ^= 1;
    }
  }
  for (int i = tid; i < P.N; i += NT) cfg[i] = S[i];
  if (tid == 0 && n_accept) {
    n_accept[(size_t)ch * PEPS_N_MOVE_TYPES + 0] += acc_h;
    n_accept[(size_t)ch * PEPS_N_MOVE_TYPES + 1] += acc_s;
  }
}

// Metropolis vertical exchanges between rows r and r+1 (two-row strip).
__global__ void __launch_bounds__(NT) k_moves2(Prob P, int r, const double* __restrict__ theta, uint8_t* configs,
                                               uint64_t seed, uint64_t gsweep, double* ws, int32_t* n_accept,
                                               int32_t* status) {
  STRIP_PROLOGUE
  build_strip(P, geo, w, r, r + 2, &one, sc);
  __syncthreads();
  int acc_v = 0;
  double* Lb[2] = {w.L, w.L + P.ES};
  double* tA = w.L + 2 * (size_t)P.ES;
  double* X0 = w.X;
  double* X1 = w.X + P.XS;
  int slot = slot_base(P, r) + P.nb_moves * (P.L2 - 1) + P.ns_moves * P.L2;
  right_envs2(P, geo, sc, S, theta, w, r);
  double rho = w.R[0];
  const double* Lc = &one;
  int cur = 0;
  for (int c = 0; c < P.L2; ++c) {
    const int i = r * P.L2 + c, j = (r + 1) * P.L2 + c;
    for (int k = 0; k < P.nb_moves; ++k, ++slot) {
      int ni, nj;
      if (!bond_proposal(P, S[i], S[j], k, ni, nj)) continue;
      lstep2(tA, Lc, sc.T[c], sc.tD[c], slice_ptr(P, geo, theta, r, c, ni), wdim(P, r, c),
             slice_ptr(P, geo, theta, r + 1, c, nj), wdim(P, r + 1, c), sc.B[c], sc.bD[c], X0, X1);
      const double rn = wg_dot(tA, w.R + (size_t)(c + 1) * P.ES, env2_size(P, sc, r, c), red);
      bool acc = false;
      if (rho == 0.0) set_status(status, PEPS_ERR_ZERO_AMPLITUDE);
      else acc = metropolis(P, rn / rho, slot_uniform(seed, ch, gsweep, slot));
      if (acc) {
        if (tid == 0) { S[i] = (uint8_t)ni; S[j] = (uint8_t)nj; }
        rho = rn;
        ++acc_v;
      }
      __syncthreads();
    }
    if (c < P.L2 - 1) {
      lstep2(Lb[cur], Lc, sc.T[c], sc.tD[c], slice_ptr(P, geo, theta, r, c, S[i]), wdim(P, r, c),
             slice_ptr(P, geo, theta, r + 1, c, S[j]), wdim(P, r + 1, c), sc.B[c], sc.bD[c], X0, X1);
      Lc = Lb[cur];
      cur ^= 1;
    }
  }
  for (int i = tid; i < P.N; i += NT) cfg[i] = S[i];
  if (tid == 0 && n_accept) n_accept[(size_t)ch * PEPS_N_MOVE_TYPES + 2] += acc_v;
}

// ---------------------------------------------------------------------------
// Measurement of row r (one-row strip): the O blocks of the row's sites, the
// local-energy terms inside the row, and (last row) log|psi| and its sign.
// epart layout per chain: [0, L1) in-row terms, [L1, 2 L1) cross-row terms,
// [2 L1] log|psi|, [2 L1 + 1] sign.
__global__ void __launch_bounds__(NT) k_meas1(Prob P, int r, const double* __restrict__ theta,
                                              const uint8_t* configs, double* ws, double* O_rows,
                                              int want_e, int32_t* status) {
  STRIP_PROLOGUE
  build_strip(P, geo, w, r, r + 1, &one, sc);
  __syncthreads();
  double* Lb[2] = {w.L, w.L + P.ES};
  double* tA = w.L + 2 * (size_t)P.ES;
  double* tB = w.L + 3 * (size_t)P.ES;
  double* X0 = w.X;
  double* X1 = w.X + P.XS;
  right_envs1(P, geo, sc, S, theta, w, r);
  const double rho = w.R[0];
  if (rho == 0.0 || !isfinite(rho)) {
    set_status(status, rho == 0.0 ? PEPS_ERR_ZERO_AMPLITUDE : PEPS_ERR_NONFINITE);
    if (tid == 0) {
      w.epart[r] = NAN;
      if (r == P.L1 - 1) { w.epart[2 * P.L1] = NAN; w.epart[2 * P.L1 + 1] = 0.0; }
    }
    return;
  }
  if (r == P.L1 - 1 && tid == 0) {
    const double ls = r >= 1 ? w.lstop[r - 1] : 0.0;
    w.epart[2 * P.L1] = ls + log(fabs(rho));
    w.epart[2 * P.L1 + 1] = rho > 0.0 ? 1.0 : -1.0;
  }
  double e = 0.0;
  double* Orow = O_rows ? O_rows + (size_t)ch * P.nnz : nullptr;
  const double* Lc = &one;
  int cur = 0;
  for (int c = 0; c < P.L2; ++c) {
    const int i = r * P.L2 + c;
    Dim4 wd = wdim(P, r, c);
    if (Orow) {
      site_env1(tA, Lc, sc.T[c], sc.tD[c], sc.B[c], sc.bD[c], w.R + (size_t)(c + 1) * P.ES, wd.n0, wd.n2, X0, X1);
      const int bs = wd.n0 * wd.n1 * wd.n2 * wd.n3;
      const double inv = 1.0 / rho;
      for (int q = tid; q < bs; q += NT) Orow[geo.ooff[i] + q] = tA[q] * inv;
      __syncthreads();
    }
    if (want_e && c < P.L2 - 1 && P.model == PEPS_MODEL_HEISENBERG) {
      for (int k = 0; k < 2; ++k) {
        int ni, nj;
        if (!bond_proposal(P, S[i], S[i + 1], k, ni, nj)) continue;
        lstep1(tA, Lc, sc.T[c], sc.tD[c], slice_ptr(P, geo, theta, r, c, ni), wd, sc.B[c], sc.bD[c], X0, X1);
        lstep1(tB, tA, sc.T[c + 1], sc.tD[c + 1], slice_ptr(P, geo, theta, r, c + 1, nj), wdim(P, r, c + 1),
               sc.B[c + 1], sc.bD[c + 1], X0, X1);
        const double rn = wg_dot(tB, w.R + (size_t)(c + 2) * P.ES, env1_size(P, sc, r, c + 1), red);
        e += 0.5 * P.J1 * (rn / rho);
      }
    }
    if (c < P.L2 - 1) {
      lstep1(Lb[cur], Lc, sc.T[c], sc.tD[c], slice_ptr(P, geo, theta, r, c, S[i]), wd, sc.B[c], sc.bD[c], X0, X1);
      Lc = Lb[cur];
      cur ^= 1;
    }
  }
  if (tid == 0) w.epart[r] = e;
}

// Cross-row local-energy terms between rows r and r+1 (two-row strip):
// vertical bonds, and next-nearest-neighbour bonds when J2 != 0.
__global__ void __launch_bounds__(NT) k_meas2(Prob P, int r, const double* __restrict__ theta,
                                              const uint8_t* configs, double* ws, int32_t* status) {
  STRIP_PROLOGUE
  build_strip(P, geo, w, r, r + 2, &one, sc);
  __syncthreads();
  double* Lb[2] = {w.L, w.L + P.ES};
  double* tA = w.L + 2 * (size_t)P.ES;
  double* tB = w.L + 3 * (size_t)P.ES;
  double* X0 = w.X;
  double* X1 = w.X + P.XS;
  right_envs2(P, geo, sc, S, theta, w, r);
  const double rho = w.R[0];
  if (rho == 0.0 || !isfinite(rho)) {
    set_status(status, rho == 0.0 ? PEPS_ERR_ZERO_AMPLITUDE : PEPS_ERR_NONFINITE);
    if (tid == 0) w.epart[P.L1 + r] = NAN;
    return;
  }
  double e = 0.0;
  const double* Lc = &one;
  int cur = 0;
  for (int c = 0; c < P.L2; ++c) {
    const int i = r * P.L2 + c, j = (r + 1) * P.L2 + c;
    if (P.model == PEPS_MODEL_HEISENBERG) {
      for (int k = 0; k < 2; ++k) {
        int ni, nj;
        if (!bond_proposal(P, S[i], S[j], k, ni, nj)) continue;
        lstep2(tA, Lc, sc.T[c], sc.tD[c], slice_ptr(P, geo, theta, r, c, ni), wdim(P, r, c),
               slice_ptr(P, geo, theta, r + 1, c, nj), wdim(P, r + 1, c), sc.B[c], sc.bD[c], X0, X1);
        const double rn = wg_dot(tA, w.R + (size_t)(c + 1) * P.ES, env2_size(P, sc, r, c), red);
        e += 0.5 * P.J1 * (rn / rho);
      }
      if (P.J2 != 0.0 && c < P.L2 - 1) {
        // bonds (r,c)-(r+1,c+1) and (r,c+1)-(r+1,c)
        for (int orient = 0; orient < 2; ++orient) {
          const int sa = orient == 0 ? i : i + 1;      // site in row r
          const int sbs = orient == 0 ? j + 1 : j;     // site in row r+1
          for (int k = 0; k < 2; ++k) {
            int na, nb;
            if (!bond_proposal(P, S[sa], S[sbs], k, na, nb)) continue;
            int s1c = S[i], s1n = S[i + 1], s2c = S[j], s2n = S[j + 1];
            if (orient == 0) { s1c = na; s2n = nb; } else { s1n = na; s2c = nb; }
            lstep2(tA, Lc, sc.T[c], sc.tD[c], slice_ptr(P, geo, theta, r, c, s1c), wdim(P, r, c),
                   slice_ptr(P, geo, theta, r + 1, c, s2c), wdim(P, r + 1, c), sc.B[c], sc.bD[c], X0, X1);
            lstep2(tB, tA, sc.T[c + 1], sc.tD[c + 1], slice_ptr(P, geo, theta, r, c + 1, s1n), wdim(P, r, c + 1),
                   slice_ptr(P, geo, theta, r + 1, c + 1, s2n), wdim(P, r + 1, c + 1), sc.B[c + 1], sc.bD[c + 1],
                   X0, X1);
            const double rn = wg_dot(tB, w.R + (size_t)(c + 2) * P.ES, env2_size(P, sc, r, c + 1), red);
            e += 0.5 * P.J2 * (rn / rho);
          }
        }
      }
    }
    if (c < P.L2 - 1) {
      lstep2(Lb[cur], Lc, sc.T[c], sc.tD[c], slice_ptr(P, geo, theta, r, c, S[i]), wdim(P, r, c),
             slice_ptr(P, geo, theta, r + 1, c, S[j]), wdim(P, r + 1, c), sc.B[c], sc.bD[c], X0, X1);
      Lc = Lb[cur];
      cur ^= 1;
    }
  }
  if (tid == 0) w.epart[P.L1 + r] = e;
}

// Diagonal energy, sum of the parts, and the per-sample outputs.
__global__ void k_finalize(Prob P, int n, const uint8_t* configs, double* ws, double* log_abs, int8_t* sign,
                           double* e_loc, int64_t out_off, int want_e, int32_t* status) {
  const int ch = blockIdx.x * blockDim.x + threadIdx.x;
  if (ch >= n) return;
  const double* ep = ws + (size_t)ch * P.chain_stride + P.off_epart;
  const uint8_t* S = configs + (size_t)ch * P.N;
  const double la = ep[2 * P.L1];
  if (log_abs) log_abs[out_off + ch] = la;
  if (sign) sign[out_off + ch] = (int8_t)ep[2 * P.L1 + 1];
  if (!isfinite(la)) set_status(status, PEPS_ERR_NONFINITE);
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
  double e = diag;
  for (int q = 0; q < 2 * P.L1 - 1; ++q) e += ep[q];
  e_loc[out_off + ch] = e;
  if (!isfinite(e)) set_status(status, PEPS_ERR_NONFINITE);
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

hipError_t launch_compress(const Prob& P, int n, int dir, int r, const double* theta, const uint8_t* configs,
                           double* ws, int32_t* status, hipStream_t st) {
  const size_t lds = compress_lds_bytes(P);
  static size_t configured = 0;
  if (lds > configured) {
    hipError_t e = hipFuncSetAttribute((const void*)k_compress, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    configured = lds;
  }
  hipLaunchKernelGGL(k_compress, dim3(n), dim3(NT), lds, st, P, dir, r, theta, configs, ws, status);
  return hipGetLastError();
}

hipError_t launch_moves1(const Prob& P, int n, int r, const double* theta, uint8_t* configs, uint64_t seed,
                         uint64_t gsweep, double* ws, int32_t* n_accept, int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_moves1, dim3(n), dim3(NT), 0, st, P, r, theta, configs, seed, gsweep, ws, n_accept, status);
  return hipGetLastError();
}

hipError_t launch_moves2(const Prob& P, int n, int r, const double* theta, uint8_t* configs, uint64_t seed,
                         uint64_t gsweep, double* ws, int32_t* n_accept, int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_moves2, dim3(n), dim3(NT), 0, st, P, r, theta, configs, seed, gsweep, ws, n_accept, status);
  return hipGetLastError();
}

hipError_t launch_meas1(const Prob& P, int n, int r, const double* theta, const uint8_t* configs, double* ws,
                        double* O_rows, int want_e, int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_meas1, dim3(n), dim3(NT), 0, st, P, r, theta, configs, ws, O_rows, want_e, status);
  return hipGetLastError();
}

hipError_t launch_meas2(const Prob& P, int n, int r, const double* theta, const uint8_t* configs, double* ws,
                        int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_meas2, dim3(n), dim3(NT), 0, st, P, r, theta, configs, ws, status);
  return hipGetLastError();
}

hipError_t launch_finalize(const Prob& P, int n, const uint8_t* configs, double* ws, double* log_abs, int8_t* sign,
                           double* e_loc, int64_t out_off, int want_e, int32_t* status, hipStream_t st) {
  const int bs = 128;
  hipLaunchKernelGGL(k_finalize, dim3((n + bs - 1) / bs), dim3(bs), 0, st, P, n, configs, ws, log_abs, sign, e_loc,
                     out_off, want_e, status);
  return hipGetLastError();
}

}  // namespace peps
