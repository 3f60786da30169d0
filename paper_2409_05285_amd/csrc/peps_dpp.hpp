// Cross-lane reductions of FP64 values inside a wavefront, built from DPP
// row permutations and the gfx950 permlane16/permlane32 swaps (no LDS
// traffic): every lane of the reduced group ends with identical bits.
#pragma once

#include <hip/hip_runtime.h>

namespace peps {

template <int CTRL>
__device__ inline double dpp_f64(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a DPP row.  Each stage adds a value and its
// mirror partner (xor 1, xor 2 in quads, then half-row and row mirrors), so
// every lane ends with the same bits.
__device__ inline double row16_sum(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);   // row_half_mirror
  v += dpp_f64<0x140>(v);   // row_mirror
  return v;
}


// Sum of the values of DPP rows 2h and 2h+1 (permlane16 swap), and of the
// two 32-lane halves (permlane32 swap).  Both lanes of a pair add the same two
// operands in the same order, so the result has identical bits on both.
__device__ inline double rows_pair_sum(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}
__device__ inline double halves_sum(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}

// Sum over the 64 lanes of a wave with identical bits on every lane, all in
// VALU cross-lane operations: mirror-pair stages inside each 16-lane row,
// then row pairs, then halves.
__device__ inline double wave_sum(double v) { return halves_sum(rows_pair_sum(row16_sum(v))); }

// N independent 16-lane row sums, stage by stage so that their latencies
// overlap.
template <int N>
__device__ inline void row16_sum_n(double* v) {
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_f64<0xB1>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_f64<0x4E>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_f64<0x141>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_f64<0x140>(v[q]);
}

// N independent wave sums, stage by stage so that their latencies overlap.
template <int N>
__device__ inline void wave_sum_n(double* v) {
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_f64<0xB1>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_f64<0x4E>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_f64<0x141>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_f64<0x140>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = rows_pair_sum(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = halves_sum(v[q]);
}

// Sum over aligned groups of g lanes inside a DPP row (g = 1, 2, 4, 8, 16;
// runtime), identical bits on every lane of the group.
__device__ inline double group_sum(double v, int g) {
  if (g >= 2) v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
  if (g >= 4) v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
  if (g >= 8) v += dpp_f64<0x141>(v);   // row_half_mirror
  if (g >= 16) v += dpp_f64<0x140>(v);  // row_mirror
  return v;
}

}  // namespace peps
