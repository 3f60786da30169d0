// Shared definitions of the HIP implementation: problem descriptor in
// device-friendly form, lattice geometry, per-chain workspace layout,
// Philox4x64-10, and deterministic workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "peps.h"

namespace peps {

constexpr int NT = 256;          // threads per workgroup of the per-chain kernels
constexpr int MAX_SITES = 256;   // L1 * L2 limit
constexpr int MAX_L = 32;        // per-dimension limit

// Problem descriptor passed by value to every kernel.
struct Prob {
  int L1, L2, N, d, d2, D, chi, model, alpha;
  int nb_moves, ns_moves, n_slots;
  double J1, J2, t, U, mu;
  int64_t nnz, np;
  // strides (in elements) of the per-chain workspace objects
  int TS;   // one boundary-MPS tensor: chi * D * chi
  int BS;   // one absorbed tensor: (chi*D) * D * (chi*D)
  int ES;   // one environment: chi * D * D * chi (two-row, also holds one-row)
  int XS;   // one contraction intermediate: chi^2 * D^3 (and >= BS)
  int64_t chain_stride;  // doubles per chain
  int64_t off_top, off_lstop, off_bot, off_lsbot, off_B, off_tmp, off_R, off_L, off_X, off_epart;
  int64_t off_top32, off_bot32;   // FP32 boundary copies (offsets in doubles)
  int64_t off_tau;                // Householder scalars of one compression [L2][chi*D]
  int64_t off_T;                  // panel T factors of the workspace-resident compression
  int64_t off_Rst;                // its R factors of every site [L2][chi D][chi D] (rebuild layout)
  int refl_store;                 // workspace-resident compression: every site's reflectors kept (1)
                                  // or rebuilt from the stored R factors (0)
  int ckernel;                    // boundary compression kernel: 1 register, 2 LDS, 3 workspace resident
  int cauto;                      // the kernel was chosen automatically (the launch may refine it by batch size)
  int mixed;                      // FP32 strip contractions
  int fermionic;                  // Z2-graded parity-even tensors (odd total parity => rho = 0)
};

// Configuration digit of site i, read through a range check: a digit
// outside [0, d^2) is read as 0 (the call's validation kernel records
// PEPS_ERR_ARG for it), so that no kernel indexes a slice out of range.
__host__ __device__ inline int digit_at(const Prob& P, const uint8_t* cfg, int i) {
  const int v = cfg[i];
  return v < P.d2 ? v : 0;
}

// Fermion-number parity of a Hubbard digit pair S = s d + s' (digit
// s = n_up + 2 n_dn): the parity of n(s) + n(s').
__host__ __device__ inline int digit_parity(const Prob& P, int S) {
  const int x = (S / P.d) ^ (S % P.d);
  return (x ^ (x >> 1)) & 1;
}

__host__ __device__ inline void leg_dims(const Prob& P, int r, int c, int& Dl, int& Du, int& Dr, int& Dd) {
  Dl = (c == 0) ? 1 : P.D;
  Du = (r == 0) ? 1 : P.D;
  Dr = (c == P.L2 - 1) ? 1 : P.D;
  Dd = (r == P.L1 - 1) ? 1 : P.D;
}

__host__ __device__ inline int block_size(const Prob& P, int r, int c) {
  int Dl, Du, Dr, Dd;
  leg_dims(P, r, c, Dl, Du, Dr, Dd);
  return Dl * Du * Dr * Dd;
}

// Per-kernel geometry tables, built in LDS by one thread at kernel start.
struct Geo {
  int poff[MAX_SITES];   // parameter offset of each site
  int ooff[MAX_SITES];   // O-row offset of each site
  // compressed boundary-MPS dims: [dir][r][c] -> (a, b); the physical leg is
  // Dd of row r (top) or Du of row r (bot).  dir 0 = top, 1 = bot.
  unsigned char ba[2][MAX_L][MAX_L];
  unsigned char bb[2][MAX_L][MAX_L];
};

// Static bond dimensions produced by the two-sweep compression of an MPS
// with input shapes (a_c, p_c, b_c): left-to-right thin QR then
// right-to-left truncation to chi.
__host__ __device__ inline void compressed_dims(int L, const int* p, int* a, int* b, int chi) {
  for (int c = 0; c < L - 1; ++c) {
    int k = a[c] * p[c] < b[c] ? a[c] * p[c] : b[c];
    b[c] = k;
    a[c + 1] = k;
  }
  for (int c = L - 1; c > 0; --c) {
    int k = chi;
    if (a[c] < k) k = a[c];
    if (p[c] * b[c] < k) k = p[c] * b[c];
    a[c] = k;
    b[c - 1] = k;
  }
}

__host__ __device__ inline void build_geo(const Prob& P, Geo& g) {
  int po = 0, oo = 0;
  for (int r = 0; r < P.L1; ++r)
    for (int c = 0; c < P.L2; ++c) {
      int i = r * P.L2 + c;
      g.poff[i] = po;
      g.ooff[i] = oo;
      int bs = block_size(P, r, c);
      po += P.d2 * bs;
      oo += bs;
    }
  int a[MAX_L], b[MAX_L], p[MAX_L];
  // top boundaries, r = 0..L1-1
  for (int c = 0; c < P.L2; ++c) { a[c] = 1; b[c] = 1; }
  for (int r = 0; r < P.L1; ++r) {
    for (int c = 0; c < P.L2; ++c) {
      int Dl, Du, Dr, Dd;
      leg_dims(P, r, c, Dl, Du, Dr, Dd);
      a[c] *= Dl;
      b[c] *= Dr;
      p[c] = Dd;
    }
    compressed_dims(P.L2, p, a, b, P.chi);
    for (int c = 0; c < P.L2; ++c) { g.ba[0][r][c] = (unsigned char)a[c]; g.bb[0][r][c] = (unsigned char)b[c]; }
  }
  for (int c = 0; c < P.L2; ++c) { a[c] = 1; b[c] = 1; }
  for (int r = P.L1 - 1; r >= 0; --r) {
    for (int c = 0; c < P.L2; ++c) {
      int Dl, Du, Dr, Dd;
      leg_dims(P, r, c, Dl, Du, Dr, Dd);
      a[c] *= Dl;
      b[c] *= Dr;
      p[c] = Du;
    }
    compressed_dims(P.L2, p, a, b, P.chi);
    for (int c = 0; c < P.L2; ++c) { g.ba[1][r][c] = (unsigned char)a[c]; g.bb[1][r][c] = (unsigned char)b[c]; }
  }
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128-bit
// multiplies with a Weyl-sequence key schedule.
struct U64x4 { uint64_t v[4]; };

__host__ __device__ inline void mulhilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
#if defined(__HIP_DEVICE_COMPILE__)
  lo = a * b;
  hi = __umul64hi(a, b);
#else
  unsigned __int128 p = (unsigned __int128)a * b;
  lo = (uint64_t)p;
  hi = (uint64_t)(p >> 64);
#endif
}

__host__ __device__ inline U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) { k0 += W0; k1 += W1; }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, hi0, lo0);
    mulhilo64(M1, c2, hi1, lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  U64x4 o;
  o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// Uniform of one proposal slot: counter (chain, sweep, slot, stream), key (seed, 0).
__host__ __device__ inline double slot_uniform(uint64_t seed, uint64_t chain, uint64_t gsweep, uint64_t slot) {
  U64x4 w = philox4x64_10(chain, gsweep, slot, 0ull, seed, 0ull);
  return (double)(w.v[0] >> 11) * 0x1.0p-53;
}

// ---------------------------------------------------------------------------
// Deterministic workgroup reduction: every thread contributes one value; the
// result (same bits on every thread) is the fixed-shape tree sum.
__device__ inline double wg_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  double out = red[0];
  __syncthreads();
  return out;
}

// Records `code` in the device status word: an error (negative code)
// replaces "fine" (0) or a warning (positive code) and is never replaced; a
// warning replaces only "fine".
__device__ inline void set_status(int32_t* status, int code) {
  if (!status) return;
  const int old = atomicCAS(status, 0, code);
  if (code < 0 && old > 0) atomicCAS(status, old, code);
}

// Singular value from a column's squared norm, for ranking the columns of a
// truncation: a non-finite norm (NaN or Inf in the data) is reported, and a
// NaN ranks last, so that the ranks still form a permutation of the columns.
__device__ inline double rank_norm(double sq, int32_t* status) {
  if (!isfinite(sq)) {
    set_status(status, PEPS_ERR_NONFINITE);
    if (sq != sq) return -1.0;
  }
  return sqrt(sq);
}

}  // namespace peps
