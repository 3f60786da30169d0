// Host-side launchers of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "peps_common.hpp"

namespace peps {

constexpr int SR_MAX_ITER = 4096;
// Largest chi * D of the workspace-resident compression kernel (its
// per-column LDS arrays), and the dynamic LDS the LDS-resident general
// kernel may use.
constexpr int CD_MAX = 512;
constexpr size_t COMPRESS_DYN_LDS_MAX = 128 * 1024;

// Bytes of the dense work matrices of the LDS-resident general kernel, and
// whether they fit its LDS.
size_t compress_dyn_lds(const Prob& P);
bool compress_in_lds(const Prob& P);
// Doubles of panel T factors one chain needs in the workspace-resident
// kernel (k_compress_big), and its launcher.
size_t compress_big_T_doubles(const Prob& P);
hipError_t launch_compress_big(const Prob& P, int n, int dir, int r, const double* theta, const uint8_t* configs,
                               double* ws, int32_t* status, hipStream_t st);
bool compress2_supported(const Prob& P);
hipError_t launch_compress2(const Prob& P, int n, int dir, int r, const double* theta, const uint8_t* configs,
                            double* ws, int32_t* status, hipStream_t st);
hipError_t launch_compress(const Prob& P, int n, int dir, int r, const double* theta, const uint8_t* configs,
                           double* ws, int32_t* status, hipStream_t st);
// Strip kernels.  theta is the FP64 parameter vector, t32 its FP32 copy
// (read instead of theta when P.mixed is set).
hipError_t launch_theta32(const Prob& P, const double* theta, float* t32, hipStream_t st);
// dst[0..n) = src[0..n) on the stream (a copy kernel: no copy or memset
// nodes when captured in a graph).
hipError_t launch_copy_bytes(uint8_t* dst, const uint8_t* src, int64_t n, hipStream_t st);
// Local values of the diagonal observables, one thread per sample.
hipError_t launch_observables(const Prob& P, int64_t n, const uint8_t* configs, double* out, hipStream_t st);
// Adds n to the device sweep counter (one thread, vector store).
hipError_t launch_advance_counter(uint64_t* ctr, uint64_t n, hipStream_t st);
hipError_t launch_moves1(const Prob& P, int n, int r, const double* theta, const float* t32, uint8_t* configs,
                         uint64_t seed, uint64_t gsweep, const uint64_t* gctr, double* ws, int32_t* n_accept,
                         int32_t* status, hipStream_t st);
hipError_t launch_moves2(const Prob& P, int n, int r, const double* theta, const float* t32, uint8_t* configs,
                         uint64_t seed, uint64_t gsweep, const uint64_t* gctr, double* ws, int32_t* n_accept,
                         int32_t* status, hipStream_t st);
// Measurement kernels (FP32 strips when P.mixed, else FP64).
hipError_t launch_meas1(const Prob& P, int n, int r, const double* theta, const float* t32, const uint8_t* configs,
                        double* ws, double* O_rows, int want_e, int32_t* status, hipStream_t st);
hipError_t launch_meas2(const Prob& P, int n, int r, const double* theta, const float* t32, const uint8_t* configs,
                        double* ws, int32_t* status, hipStream_t st);
// Mixed precision: FP64 measurement of the row strips in `list` (device:
// count, then items chain * 64 + kind), one persistent launch.
hipError_t launch_remeasure(const Prob& P, int n, const double* theta, const uint8_t* configs, double* ws,
                            const int32_t* list, double* O_rows, int want_e, int32_t* status, hipStream_t st);
hipError_t launch_finalize(const Prob& P, int n, const uint8_t* configs, double* ws, double* log_abs, int8_t* sign,
                           double* e_loc, int64_t out_off, int want_e, int redo, int32_t* status, hipStream_t st);
// Mixed precision: the row strips of the samples to measure again in FP64
// (masks per sample) and their list (list[0] = count, then the items).
hipError_t launch_redo_flags(const Prob& P, int n, double* ws, int want_e, int32_t* list, hipStream_t st);
// PEPS_ERR_ARG in status if a digit of configs [n][N] is >= d^2.
hipError_t launch_check_digits(const Prob& P, int64_t n, const uint8_t* configs, int32_t* status, hipStream_t st);
// Weighted means and standard errors of per-sample quantities.
hipError_t launch_sample_stats(const Prob& P, int n_sweeps, int n_chains, int k, const double* values,
                               const double* weights, const double* log_abs, double* out, hipStream_t st);

// Simple update (spin-1/2 Heisenberg, J2 = 0, D <= MAX_SU_D): one Trotter
// step of tau over the four bond groups; sqrt(lambda) absorbed into theta.
constexpr int MAX_SU_D = 8;
size_t su_bond_doubles(const Prob& P);
int su_max_group(const Prob& P);
hipError_t launch_su_step(const Prob& P, double* theta, double* lam, double tau, double* ws, int32_t* status,
                          hipStream_t st);
hipError_t launch_su_absorb(const Prob& P, const double* theta, const double* lam, double* out, hipStream_t st);

// Direct sampling (Appendix A): per-chain scratch of the draw kernel
// (offsets and stride in doubles), built from the chain problem P and the
// double layer's problem Q (d^2 = 1, bond D^2, boundary chi_dl).
struct DirectLayout {
  int64_t TDS, ENV;   // one doubled top tensor; one left / right environment
  int64_t off_td, off_R, off_L, off_X0, off_X1, off_env, off_Px, stride;
  int64_t x1;         // largest strip intermediate (doubles)
};
DirectLayout direct_layout(const Prob& P, const Prob& Q);
// E_i = sum_S T_i[S] (x) T_i[S] into eth (Q's parameter layout); clears cfg_q [N].
hipError_t launch_double_layer(const Prob& P, const Prob& Q, const double* theta, double* eth, uint8_t* cfg_q,
                               hipStream_t st);
// Row r of every chain's draw (conditionals, inverse-CDF pick, log p).
hipError_t launch_direct_row(const Prob& P, const Prob& Q, const DirectLayout& L, int n, int r, const double* theta,
                             const double* eth, uint8_t* configs, double* ws, const double* wsq, double* dws,
                             uint64_t seed, uint64_t draw, int reweight, const double* b_diag, double* log_p,
                             int32_t* status, hipStream_t st);
hipError_t launch_update_b(const Prob& P, int n, const uint8_t* configs, double* b_diag, hipStream_t st);
hipError_t launch_importance_weights(int64_t n, const double* log_abs, const double* log_p, double* w,
                                     hipStream_t st);

size_t sr_workspace_bytes(const Prob& P, int64_t n_s);
// Bytes of the fixed per-GPU scratch of sr_cg_solve_noalloc, and its device
// address on the current device (resolved once per device; nullptr if the
// symbol cannot be resolved).
constexpr size_t SR_STATIC_BYTES = (size_t)PEPS_SR_STATIC_BYTES;
void* sr_static_scratch();
hipError_t launch_sr(const Prob& P, int64_t n_s, const uint8_t* configs, const double* O, const double* weights,
                     const double* log_abs, const double* e_loc, double tau, double eps, int max_iter, double rtol, double* dtheta,
                     double* g_out, double* theta, double* stats, int32_t* status, void* ws, hipStream_t st);
hipError_t launch_vjp(const Prob& P, int64_t n_s, const uint8_t* configs, const double* O, const double* cot,
                      double* grad, void* ws, hipStream_t st);

}  // namespace peps
