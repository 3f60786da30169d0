// Per-chain workspace views, strip boundaries, slice pointers and the
// Metropolis proposal set, shared by the chain kernels.
#pragma once

#include "peps_common.hpp"
#include "peps_contract.hpp"

namespace peps {

struct ChainWS {
  double *top, *lstop, *bot, *lsbot, *B, *tmp, *R, *L, *X, *epart;
  float *top32, *bot32;   // FP32 copies of the boundaries (mixed precision)
};

// Per-chain measurement record (epart), in doubles:
//   [0, L1)            in-row local-energy terms of each row,
//   [L1, 2 L1)         cross-row terms of each row pair,
//   [2 L1], [2 L1 + 1] log|psi| and its sign,
//   mixed precision only, three values per row (epart_err1 + 3 r, one-row
//   strips) and per row pair (epart_err2 + 3 r, two-row strips): the largest
//   relative deviation of the strip amplitude recomputed at the column cuts,
//   the largest u32-weighted cancellation of those cut dot products, and the
//   sum over the row's local-energy terms of |coef rho(S') / rho|,
//   [8 L1 + 2]            re-measure flag: 0 none, 1 some strips for the
//                         local energy only, 2 some one-row strips with
//                         their O rows too,
//   [8 L1 + 3]            the FP32 pass's local energy, [8 L1 + 4] its
//                         error estimate,
//   [8 L1 + 5 .. 8 L1 + 7] bit masks of the strips measured again in FP64:
//                         one-row strips with their O rows (bit r), one-row
//                         strips, two-row strips (bit r: rows r, r + 1).
__host__ __device__ inline int epart_err1(const Prob& P) { return 2 * P.L1 + 2; }
__host__ __device__ inline int epart_err2(const Prob& P) { return 5 * P.L1 + 2; }
__host__ __device__ inline int epart_flag(const Prob& P) { return 8 * P.L1 + 2; }
__host__ __device__ inline int epart_e32(const Prob& P) { return 8 * P.L1 + 3; }
__host__ __device__ inline int epart_mask(const Prob& P) { return 8 * P.L1 + 5; }
__host__ __device__ inline int epart_size(const Prob& P) { return 8 * P.L1 + 8; }

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
  w.top32 = (float*)(base + P.off_top32);
  w.bot32 = (float*)(base + P.off_bot32);
  return w;
}

// Boundary tensors of one precision.
template <typename T> __device__ inline T* top_of(const ChainWS& w);
template <> __device__ inline double* top_of<double>(const ChainWS& w) { return w.top; }
template <> __device__ inline float* top_of<float>(const ChainWS& w) { return w.top32; }
template <typename T> __device__ inline T* bot_of(const ChainWS& w);
template <> __device__ inline double* bot_of<double>(const ChainWS& w) { return w.bot; }
template <> __device__ inline float* bot_of<float>(const ChainWS& w) { return w.bot32; }

// Boundary tensors and dimensions of the strip around row r (one-row:
// top[r-1] and bot[r+1]; two-row: top[r-1] and bot[r+2]), with the
// trivial boundary (one element equal to 1) outside the lattice.
template <typename T>
struct StripCtx {
  const T* T_[MAX_L];
  const T* B[MAX_L];
  Dim3 tD[MAX_L];
  Dim3 bD[MAX_L];
};

template <typename T>
__device__ inline void build_strip(const Prob& P, const Geo& g, const ChainWS& w, int r, int rb, const T* one,
                                   StripCtx<T>& s) {
  if (threadIdx.x != 0) return;
  const T* top = top_of<T>(w);
  const T* bot = bot_of<T>(w);
  for (int c = 0; c < P.L2; ++c) {
    int Dl, Du, Dr, Dd;
    leg_dims(P, r, c, Dl, Du, Dr, Dd);
    if (r >= 1) {
      s.T_[c] = top + ((size_t)(r - 1) * P.L2 + c) * P.TS;
      s.tD[c] = Dim3{g.ba[0][r - 1][c], Du, g.bb[0][r - 1][c]};
    } else {
      s.T_[c] = one;
      s.tD[c] = Dim3{1, 1, 1};
    }
    if (rb <= P.L1 - 1) {
      int Dl2, Du2, Dr2, Dd2;
      leg_dims(P, rb, c, Dl2, Du2, Dr2, Dd2);
      s.B[c] = bot + ((size_t)rb * P.L2 + c) * P.TS;
      s.bD[c] = Dim3{g.ba[1][rb][c], Du2, g.bb[1][rb][c]};
    } else {
      s.B[c] = one;
      s.bD[c] = Dim3{1, 1, 1};
    }
  }
}

template <typename T>
__device__ inline const T* slice_ptr(const Prob& P, const Geo& g, const T* theta, int r, int c, int S) {
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

// Spin exchange S^+_a S^-_b + S^-_a S^+_b on one side (0: ket digits, 1: bra
// digits) of two sites: the exchanged configuration, or false when the term
// vanishes.  Heisenberg: the two spins differ.  Hubbard (digit n_up + 2 n_dn):
// both sites singly occupied with opposite spins; the two on-site bilinears
// c^dag_up c_dn act on adjacent Jordan-Wigner modes, so the term carries no
// sign.
__device__ inline bool spin_exchange(const Prob& P, int Sa, int Sb, int side, int& na, int& nb) {
  const int a = side == 0 ? ket_of(P, Sa) : bra_of(P, Sa);
  const int b = side == 0 ? ket_of(P, Sb) : bra_of(P, Sb);
  if (a == b) return false;
  if (P.model == PEPS_MODEL_HUBBARD && (a == 0 || a == 3 || b == 0 || b == 3)) return false;
  na = side == 0 ? merge(P, b, bra_of(P, Sa)) : merge(P, ket_of(P, Sa), b);
  nb = side == 0 ? merge(P, a, bra_of(P, Sb)) : merge(P, ket_of(P, Sb), a);
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

// Jordan-Wigner sign of moving the sigma particle of one side (0: ket digit,
// 1: bra digit) between sites i and j: modes are numbered 2 site + sigma
// (sites row-major, up before down), and the sign is -1 to the number of
// occupied modes strictly between the two.
__device__ inline double jw_sign(const Prob& P, const uint8_t* S, int side, int i, int j, int sg) {
  int lo = 2 * i + sg, hi = 2 * j + sg;
  if (lo > hi) { const int t = lo; lo = hi; hi = t; }
  int cnt = 0;
  for (int m = lo + 1; m < hi; ++m) {
    const int dg = side == 0 ? ket_of(P, S[m >> 1]) : bra_of(P, S[m >> 1]);
    cnt += (dg >> (m & 1)) & 1;
  }
  return (cnt & 1) ? -1.0 : 1.0;
}

// Coefficient of the off-diagonal term of calH reached by bond proposal k
// (Heisenberg: J/2; Hubbard: -t times the Jordan-Wigner sign).
__device__ inline double bond_coeff(const Prob& P, const uint8_t* S, int i, int j, int k, double J) {
  if (P.model == PEPS_MODEL_HEISENBERG) return 0.5 * J;
  return -P.t * jw_sign(P, S, k / 2, i, j, k % 2);
}

__device__ inline bool metropolis(const Prob& P, double R, double u) {
  double wgt = P.alpha == 2 ? R * R : fabs(R);
  return u < fmin(1.0, wgt);
}

}  // namespace peps
