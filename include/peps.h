/*
 * peps.h -- C ABI of the MI355X thermal PEPS-VMC hot path.
 *
 * The method (arXiv 2409.05285, Method section): the thermal density matrix
 * is vectorised (Eq. 2) into a PEPS with one merged physical index
 * S_i = (s_i, s'_i) of dimension d^2 per site (Eq. 4), sampled by Markov-chain
 * Monte Carlo with weight |rho_theta(S)|^2, evaluated per sample through
 * boundary-MPS contraction of the single-layer network (boundary dimension
 * chi, the paper's D_c), and cooled from beta = 0 by stochastic
 * reconfiguration: (S + eps 1) dtheta = -tau g, solved by conjugate gradient
 * with the separable metric (Eqs. 5-10).
 *
 * Conventions shared by every call
 *   site (r, c), r = 0..L1-1 (top to bottom), c = 0..L2-1, i = r*L2 + c;
 *   theta: sites in order i, each a block T_i[S][l][u][r][d] (row-major,
 *     d^2 slices; a virtual leg that leaves the open lattice has dimension 1,
 *     the others D); N_p = peps_param_count();
 *   configuration: uint8 S_i = s*d + s' per site, [n][L1*L2];
 *   O row of one sample: sites in order i, each a [l][u][r][d] block holding
 *     d log rho / d T_i[S_i] (the other d^2-1 slices of the site are zero and
 *     not stored); nnz = peps_orow_count();
 *   spin digit s: 0 = up, 1 = down.  Hubbard digit s = n_up + 2 n_dn;
 *     fermion modes are numbered 2 i + sigma (sites row-major, up before
 *     down), and a hop between modes a and b carries the Jordan-Wigner sign
 *     (-1)^(occupied modes strictly between a and b), taken in the ket digits
 *     for the H (x) 1 half of calH and in the bra digits for 1 (x) H^T.  The
 *     tensors are plain (no fermionic swap signs in the contraction).
 *
 * Memory and streams.  Every pointer argument of the device calls is a
 * device pointer unless stated otherwise; the caller owns all memory,
 * including the workspace sized by peps_workspace_bytes().  Device calls
 * enqueue on `stream` and return without synchronising; they allocate and
 * free nothing.  Calls that share one workspace must not overlap.
 *
 * Errors.  Shape and argument errors are returned before anything is
 * enqueued.  A failed launch returns PEPS_ERR_HIP.  Data-dependent failures
 * (non-finite parameters, a zero amplitude, CG breakdown, a configuration
 * digit outside [0, d^2)) are recorded in the device word `status` (0 =
 * fine, otherwise a peps_status value; the first error wins), which the
 * caller reads after its own synchronisation.  Digits are read only after
 * a range check: a digit >= d^2 records PEPS_ERR_ARG and is read as 0, so
 * that no kernel indexes theta or a parameter vector out of range (the
 * results of such a sample are then meaningless).
 */
#ifndef PEPS_H
#define PEPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* peps_stream_t; /* a hipStream_t */

typedef enum {
  PEPS_OK = 0,
  PEPS_ERR_ARG = -1,         /* bad shape, null pointer, out-of-range value   */
  PEPS_ERR_UNSUPPORTED = -2, /* valid but beyond the compiled tile limits     */
  PEPS_ERR_HIP = -3,         /* a HIP runtime call or launch failed           */
  PEPS_ERR_WORKSPACE = -4,   /* ws_bytes smaller than peps_workspace_bytes()  */
  PEPS_ERR_NONFINITE = -5,   /* NaN / Inf met in the data (device status)     */
  PEPS_ERR_ZERO_AMPLITUDE = -6, /* a strip amplitude of a sample is exactly 0 */
  PEPS_ERR_CG_BREAKDOWN = -7,   /* p^T A p <= 0 in conjugate gradient         */
  PEPS_WARN_CG_NOT_CONVERGED = 1
} peps_status;

enum { PEPS_MODEL_HEISENBERG = 0, PEPS_MODEL_HUBBARD = 1 };
enum { PEPS_PREC_FP64 = 0, PEPS_PREC_MIXED = 1 };
enum { PEPS_WS_EVAL = 0, PEPS_WS_GRAD = 1, PEPS_WS_SWEEP = 2, PEPS_WS_SR = 3, PEPS_WS_SU = 4,
       PEPS_WS_MIN = 5 };
enum { PEPS_N_MOVE_TYPES = 3 }; /* horizontal exchange, site move, vertical exchange */
enum { PEPS_N_OBS = 4 };        /* local values per sample of peps_observables_batch */

typedef struct {
  int32_t L1, L2;    /* rows, columns (open boundaries), each >= 2                */
  int32_t d;         /* single-copy local dimension: 2 spin-1/2, 4 Hubbard        */
  int32_t D, chi;    /* PEPS bond dimension; boundary-MPS dimension (D_c)          */
  int32_t model;     /* PEPS_MODEL_*                                               */
  double J1, J2;     /* Heisenberg couplings (Benchmark section, Eq. j1j2eq).  On
                        the Hubbard lattice J2 adds J2 sum_<<ij>> S_i.S_j over
                        next-nearest-neighbour pairs (S^z = (n_up - n_dn)/2,
                        S^+ = c^dag_up c_dn; no Jordan-Wigner sign); 0 gives the
                        plain Hubbard model                                      */
  double t, U, mu;   /* Hubbard parameters (Benchmark section, Eq. hubbard_model)  */
  int32_t precision; /* PEPS_PREC_*: FP64 throughout, or FP32 strip contractions
                        with FP64 truncation / reductions / log-scales.  In the
                        mixed form every row strip of a measurement also
                        estimates its own rounding error; a one-row strip
                        whose amplitude estimate exceeds 3e-5 (relative) is
                        measured again with the FP64 strips together with its
                        O rows (and log|psi| and the sign when it is the last
                        row), and then, while a sample's local-energy estimate
                        over its remaining FP32 strips exceeds 5e-5 max(|E_loc|,
                        mean |E_loc| of the call's batch), its strip of largest
                        contribution is measured again for the energy.
                        Metropolis ratios stay FP32.                          */
  int32_t alpha;     /* sampling weight |rho|^alpha: 2, or 1 (Appendix A, Eq. A1)  */
  int32_t fermionic; /* 0: plain tensors.  1 (Hubbard only): the tensors are
                        Z2-graded and parity-even (Method section, fPEPS
                        paragraph): every site tensor is nonzero only where
                        p(S) + p(l) + p(u) + p(r) + p(d) is even, p(S) the
                        fermion-number parity of the digits (s, s') and a bond
                        index even for index < D/2.  A configuration of odd
                        total parity then has amplitude exactly 0; the device
                        decides it from the digits in integer arithmetic and
                        reports it as a zero amplitude without contracting     */
  int32_t compress_kernel; /* PEPS_COMPRESS_*: which kernel runs the boundary
                        row compression.  AUTO (0): the register-resident one
                        where its limits allow (chi D <= 64, D in {1, 2, 4}),
                        except for calls on 512 or more chains with
                        chi D^2 <= 64, which take the LDS-resident one; else
                        the LDS-resident one where its matrices fit 128 KB,
                        else the workspace-resident one.  REGISTER,
                        LDS or WORKSPACE force one; a kernel whose limits the
                        shape exceeds is PEPS_ERR_UNSUPPORTED.  All compute
                        the same compression (Method section, boundary MPS
                        with D_c = chi) and agree to rounding; the workspace
                        layout (peps_workspace_bytes) follows the choice.
                        See peps_autotune_compression.                        */
} peps_desc;

enum { PEPS_COMPRESS_AUTO = 0, PEPS_COMPRESS_REGISTER = 1, PEPS_COMPRESS_LDS = 2, PEPS_COMPRESS_WORKSPACE = 3 };

/* Instrumentation handle (not part of the method): a caller-owned record of
   HIP event pairs around the kernel launches of the device calls that
   receive it.  NULL everywhere means no instrumentation.  A trace is used by
   one stream at a time; the library keeps no state of its own. */
typedef struct peps_trace peps_trace;

/* ---- host, pure ------------------------------------------------------- */

/* N_p: total number of parameters (Method section: theta_1..theta_{N_p}).
   Returns -1 for an invalid descriptor. */
int64_t peps_param_count(const peps_desc* desc);

/* Entries stored per O row (one [l][u][r][d] block per site). -1 if invalid. */
int64_t peps_orow_count(const peps_desc* desc);

/* Proposal slots per sweep (each owns one uniform). -1 if invalid. */
int64_t peps_slot_count(const peps_desc* desc);

/* Workspace bytes for `what` = PEPS_WS_EVAL / _GRAD / _SWEEP (n = number of
   chains or samples), PEPS_WS_SR (n = number of samples N_s), PEPS_WS_SU,
   or PEPS_WS_MIN: the smallest workspace an evaluation, gradient or sweep
   call on n chains accepts.  The two differ only where chi * D > 64 and the
   QR matrices do not fit on chip: the full size keeps every site's QR
   reflectors of a boundary compression; with less (down to PEPS_WS_MIN) the
   compression keeps only the R factors and rebuilds each site's reflectors
   when the truncation sweep needs them (same results bit for bit, about a
   quarter more compression time, an eighth of that memory at 16x16,
   chi = 64, D = 8). */
peps_status peps_workspace_bytes(const peps_desc* desc, int64_t n, int32_t what, size_t* bytes);

/* Static text for a status code. */
const char* peps_status_string(peps_status s);

/* ---- device ------------------------------------------------------------- */

/* Fixed-configuration evaluation (Method section, Eqs. 8-9 and in_en).
   For each of the n configurations: log|psi| = log|rho_{L1-1}(S)| (the
   top-down boundary-MPS amplitude), its sign (+1/-1) and the local energy
   E_loc(S) = sum_S' calH_{SS'} rho(S')/rho(S) with calH = H(x)I + I(x)H^T
   (Eq. 3), ratios taken from one-row strips (terms inside a row) or
   two-row strips (terms across rows).
   configs [n][N] uint8; log_abs [n] f64; sign [n] int8; e_loc [n] f64
   (e_loc may be NULL); status: one device int32.  A sample whose amplitude
   is exactly zero gets log_abs = -inf, sign 0 and an undefined (NaN) local
   energy, and the status records PEPS_ERR_ZERO_AMPLITUDE; non-finite data
   give NaN and PEPS_ERR_NONFINITE (the first error of a call is kept). */
peps_status peps_eval_batch(const peps_desc* desc, const double* theta, int32_t n,
                            const uint8_t* configs, double* log_abs, int8_t* sign,
                            double* e_loc, int32_t* status, void* ws, size_t ws_bytes,
                            peps_trace* trace, peps_stream_t stream);

/* Log-derivatives O_k(S) = d rho / d theta_k / rho (Method section, Eq. 8)
   of n fixed configurations, one compressed row each: O_rows [n][nnz] f64.
   The block of site (r, c) is the derivative of the one-row strip rho_r with
   the boundaries top[r-1], bot[r+1] held fixed (they do not depend on row r).
   log_abs may be NULL. */
peps_status peps_grad_batch(const peps_desc* desc, const double* theta, int32_t n,
                            const uint8_t* configs, double* O_rows, double* log_abs,
                            int32_t* status, void* ws, size_t ws_bytes, peps_trace* trace,
                            peps_stream_t stream);

/* n_sweeps Metropolis sweeps of n_chains independent chains (Method section:
   MCMC over S; acceptance min(1, |R|^alpha)), each sweep followed by a
   measurement of the final configuration.
   Sweep order per row r: horizontal exchanges (ket then bra digit) on bonds
   c = 0..L2-2 with one-row strip ratios; site moves c = 0..L2-1; if r < L1-1
   vertical exchanges c = 0..L2-1 with two-row strip ratios; then the top
   boundary of row r is recomputed.  The uniform of proposal slot q in global
   sweep g of chain ch is Philox4x64-10 with counter (ch, g, q, 0) and key
   (seed, 0): u = (w0 >> 11) * 2^-53; sweep k of this call has
   g = sweep0 + c + k, where c = *sweep_counter (read on the device) when
   sweep_counter is not NULL, else 0.  sweep_counter: one device uint64 or
   NULL; when given, the call adds n_sweeps to it after its last kernel, so a
   call captured once in a HIP graph draws fresh uniforms on every replay.
   configs [n_chains][N] in/out.  Per sweep k and chain ch (index k*n_chains+ch):
   log_abs, sign, e_loc [n_sweeps*n_chains], O_rows [n_sweeps*n_chains][nnz];
   any of these may be NULL (then not written).  sample_configs
   [n_sweeps*n_chains][N] uint8 (may be NULL) receives the configuration each
   measurement was taken on, the row order of O_rows, so that the samples of
   several sweeps can go to sr_cg_solve together.  n_accept [n_chains][3]
   int32 is incremented by the accepted moves of each type (may be NULL). */
peps_status peps_sample_sweep(const peps_desc* desc, const double* theta, int32_t n_chains,
                              uint8_t* configs, uint64_t seed, uint64_t sweep0,
                              uint64_t* sweep_counter, int32_t n_sweeps, double* log_abs,
                              int8_t* sign, double* e_loc, double* O_rows, uint8_t* sample_configs,
                              int32_t* n_accept, int32_t* status, void* ws, size_t ws_bytes,
                              peps_trace* trace, peps_stream_t stream);

/* Stochastic-reconfiguration update (Method section, Eqs. 5-7 and 10):
   Ebar = <E>, obar = <O>, g = <O (E - Ebar)>, S x = <O (O.x - obar.x)>,
   and (S + eps 1) dtheta = -tau g solved by conjugate gradient from
   dtheta = 0, never forming S: each iteration applies O (gather) then O^T
   (scatter).  The averages <f> = sum_i w_i f_i / sum_i w_i take their
   weights from, in this order: `weights` [n_s] when not NULL; else, when
   `log_abs` [n_s] is not NULL, w_i = |rho_i|^(2 - alpha) formed on the
   device from the log-amplitudes (relative to their largest, so no value
   overflows): uniform for alpha = 2, and |rho_i| for samples drawn from
   |rho| (alpha = 1, Appendix A, Eq. A1); else uniform.  The residual test
   ||r|| <= rtol ||b|| (b = -tau g) is taken before each iteration; at most
   max_iter iterations.
   configs [n_s][N] uint8; O_rows [n_s][nnz]; e_loc [n_s];
   dtheta [N_p] out; g_out [N_p] out or NULL; theta [N_p] in/out or NULL:
   when given, the update theta <- theta + dtheta (Eq. 5) is applied too;
   stats [PEPS_SR_NSTATS] device f64 out: Ebar, final ||r||, iterations,
   ||b||, and 1 if the solve stopped at max_iter with ||r|| > rtol ||b||
   (else 0).  That case also records PEPS_WARN_CG_NOT_CONVERGED in `status`
   when no error is recorded there (a warning never replaces an error; an
   error replaces a warning).  CG breakdown is reported in `status` (theta
   is then left unchanged). */
enum { PEPS_SR_NSTATS = 5 };
peps_status sr_cg_solve(const peps_desc* desc, int64_t n_s, const uint8_t* configs,
                        const double* O_rows, const double* weights, const double* log_abs,
                        const double* e_loc, double tau, double eps, int32_t max_iter, double rtol,
                        double* dtheta, double* g_out, double* theta, double* stats,
                        int32_t* status, void* ws, size_t ws_bytes, peps_trace* trace,
                        peps_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc):
   sr_cg_solve without a workspace argument, same arguments, results and
   kernels otherwise.  Its scratch is one fixed device array of
   PEPS_SR_STATIC_BYTES per GPU, reserved when the library's code is loaded
   on that GPU and held until the process ends; its address is resolved on
   the first call on each device (with that device current).  A call whose
   scratch need, peps_workspace_bytes(desc, n_s, PEPS_WS_SR), exceeds that
   size returns PEPS_ERR_WORKSPACE before anything is enqueued (64 MiB holds
   the 8x8, D = 4 solve on 204,800 samples and the 12x12, D = 6 one on 4096).
   The call allocates and frees nothing.  Every call on one GPU uses that
   GPU's array, which keeps the last call's contents (the solve writes every
   entry it reads before reading it): calls that overlap on one GPU (other
   streams, other threads) race and must be serialised by the caller. */
enum { PEPS_SR_STATIC_BYTES = 64 << 20 };
peps_status sr_cg_solve_noalloc(const peps_desc* desc, int64_t n_s, const uint8_t* configs,
                                const double* O_rows, const double* weights, const double* log_abs,
                                const double* e_loc, double tau, double eps, int32_t max_iter, double rtol,
                                double* dtheta, double* g_out, double* theta, double* stats,
                                int32_t* status, peps_stream_t stream);

/* Sample statistics of k per-sample quantities (Method section: the
   averages of Eqs. 6-7 and in_en; Appendix A, Eq. A1 for alpha = 1):
   values [n_sweeps * n_chains][k] f64, sample index i = sweep * n_chains +
   chain (the row order of peps_sample_sweep's outputs).  Weights as in
   sr_cg_solve: `weights` [n_sweeps * n_chains] when not NULL, else
   |rho_i|^(2 - alpha) from log_abs when it is not NULL, else uniform.
   out [k][2] f64: the weighted mean over all samples, and the standard
   error of the mean estimated from the n_chains per-chain weighted means
   (their sample standard deviation over sqrt(n_chains); 0 when n_chains =
   1).  One kernel, fixed summation order; no workspace. */
peps_status peps_sample_stats(const peps_desc* desc, int32_t n_sweeps, int32_t n_chains, int32_t k,
                              const double* values, const double* weights, const double* log_abs,
                              double* out, peps_stream_t stream);

/* Vector-Jacobian product of the log-amplitudes (Eq. 8: O_i is the gradient
   of log|rho(S_i)| with respect to theta): grad = sum_i cot_i O_i, scattered
   from the compressed O rows into the parameter layout.  This is the
   backward pass of theta -> log|psi| on a batch of configurations.
   configs [n][N] uint8; O_rows [n][nnz] (from peps_grad_batch or
   peps_sample_sweep); cot [n] f64; grad [N_p] f64 out (overwritten).
   Workspace: peps_workspace_bytes(desc, n, PEPS_WS_SR). */
peps_status peps_vjp_batch(const peps_desc* desc, int64_t n, const uint8_t* configs, const double* O_rows,
                           const double* cot, double* grad, void* ws, size_t ws_bytes, peps_stream_t stream);

/* Local values of diagonal thermal observables (Benchmark section: uniform
   susceptibility chi = beta <M_z^2> / N with <M_z>^2 taken as 0; double
   occupancy of the Hubbard model).  For an operator A diagonal in the
   computational basis the local value of sample S = (s, s') is
   (A(s) + A(s')) / 2, whose |rho|^2-weighted mean is the symmetrised
   expectation Tr(rho rho^T A + rho^T rho A) / (2 Tr(rho rho^T)).
   out [n][PEPS_N_OBS] f64, per sample: M_z, M_z^2, particle number (Hubbard;
   0 for spins), double occupancy sum_i n_i,up n_i,dn (Hubbard; 0 for spins),
   with S^z = 1/2 - s for spins and (n_up - n_dn) / 2 for Hubbard.  The values
   are exact multiples of 1/8.  configs [n][N] uint8.  Enqueues one kernel;
   no workspace.  Off-diagonal correlations such as sum S_i.S_j over a bond
   set are local energies of a Hamiltonian with those couplings (J1, J2 of
   peps_desc; peps_eval_batch), halved: with J2 = 1 and every other coupling
   0 (J1 = 0; Hubbard t = U = mu = 0) the mean local energy over 2 M is the
   next-nearest-neighbour spin correlation F of the Benchmark section, M the
   number of such pairs. */
peps_status peps_observables_batch(const peps_desc* desc, int64_t n, const uint8_t* configs, double* out,
                                   peps_stream_t stream);

/* Simple-update imaginary-time evolution, the paper's alternative to SR at
   the highest temperatures (the paragraph on the simple-update method after
   Appendix A; the scheme of Jiang, Weng and Xiang): n_steps first-order
   Trotter steps of tau, each applying exp(-tau calH_b) = exp(-tau J1 h) (x)
   exp(-tau J1 h), h = S_i.S_j, to every nearest-neighbour bond in four groups
   of disjoint bonds (horizontal bonds with c even, c odd; vertical bonds with
   r even, r odd), with bond weights lambda standing in for the environment.
   One step of tau evolves like one SR step of tau (beta_phys = 4 n tau).  Per
   bond: the other legs of both sites are multiplied by their weights, the
   two-site tensor gets the gate and an SVD, the D largest values are kept
   (lambda_b = kept / largest), and the other legs are divided by their
   weights again (a weight at or below 1e-12 of its bond's largest counts as
   zero).  theta [N_p] and lambdas [n_bonds][D] f64 are updated in place;
   n_bonds = L1 (L2-1) + (L1-1) L2, horizontal bonds row-major first, then
   vertical bonds row-major; start from lambdas = 1.  Spin-1/2 Heisenberg
   with J2 = 0 and D <= 8 only (else PEPS_ERR_UNSUPPORTED).  ws: at least
   peps_workspace_bytes(desc, 0, PEPS_WS_SU).  Non-finite singular values
   are reported in status. */
peps_status peps_simple_update(const peps_desc* desc, double* theta, double* lambdas, double tau, int32_t n_steps,
                               int32_t* status, void* ws, size_t ws_bytes, peps_stream_t stream);

/* The plain PEPS of a simple-update state: theta_out = theta with
   sqrt(lambda_b) multiplied into both ends of every bond (the input of
   sampling and SR).  theta_out [N_p] may not alias theta. */
peps_status peps_su_absorb(const peps_desc* desc, const double* theta, const double* lambdas, double* theta_out,
                           peps_stream_t stream);

/* ---- launch tuning -------------------------------------------------------- */

/* Host call (synchronises `stream`): times the boundary compression of n
   chains' configurations with every compression kernel valid for desc's
   shape (desc->compress_kernel is ignored): per candidate one untimed pass,
   then `repeats` passes, each computing the top and the bottom boundaries
   of every row, timed by HIP events.  ms[k] for k = PEPS_COMPRESS_REGISTER,
   _LDS, _WORKSPACE (ms[0] unused) receives the mean milliseconds per pass,
   or -1 where the kernel does not apply; *best the fastest.  ms [4] and
   best are host pointers.  theta, configs, status, ws: as for
   peps_eval_batch, with ws_bytes at least the largest of
   peps_workspace_bytes(desc with compress_kernel = k, n, PEPS_WS_EVAL) over
   the valid k (PEPS_ERR_WORKSPACE otherwise).  repeats in [1, 100]. */
peps_status peps_autotune_compression(const peps_desc* desc, const double* theta, int32_t n, const uint8_t* configs,
                                      int32_t repeats, double* ms, int32_t* best, int32_t* status, void* ws,
                                      size_t ws_bytes, peps_stream_t stream);

/* ---- direct sampling (Appendix A, Eqs. A2-A7) -------------------------- */

/* Workspace bytes of peps_direct_sample for n_chains chains and double-layer
   boundary dimension chi_dl.  PEPS_ERR_UNSUPPORTED where one of the draw
   kernel's per-chain intermediates (sized from the actual bond dimensions;
   up to D^6 chi^2 chi_dl doubles in the bulk) exceeds 2^24 doubles or
   chi_dl D^2 exceeds the compression kernels' 512. */
peps_status peps_direct_workspace_bytes(const peps_desc* desc, int64_t n_chains, int32_t chi_dl, size_t* bytes);

/* Direct (autoregressive) sampling (Appendix A, Eqs. A2-A6): every chain
   draws one configuration, sites row-major, each from its conditional
   probability given the sites drawn before it,
     p_2c(S_i | S_<i) proportional to the sum of |rho(S)|^2 over S_>i
   (reweight = 0), or p_4c = b(S_i) sqrt(p_2c) normalised over S_i
   (reweight = 1; b = 1 where s_i != s'_i, b = *b_diag where s_i = s'_i).
   The marginals are those of the double-layer network sum_S rho(S)^2: site
   tensors E_i = sum_S T_i[S] (x) T_i[S] (legs of dimension D^2), whose bottom
   boundaries are compressed to chi_dl by the row compression of the
   single-layer path; the rows already drawn enter as their single-layer top
   boundary (compressed to desc->chi on the drawn digits) paired with
   itself.  A negative marginal (truncation) counts as 0.  With chi_dl and
   chi large enough to truncate nothing, the draw is exact: p_2(S) =
   |rho(S)|^2 / Z.  Site i of chain c takes the uniform of Philox4x64-10 with
   counter (c, draw, i, 3) and key (seed, 0) and picks the first digit whose
   running sum of probabilities (digit order) exceeds it.
     configs [n_chains][N] u8 (out); log_p [n_chains] f64 (out): log of the
   probability the sampler gave the drawn configuration (the product of the
   conditionals it used), the denominator of the importance weight
   r = |rho|^2 / p (Eq. A7; see peps_importance_weights).  b_diag: device
   pointer to one f64, read when reweight = 1; with update_b = 1 it is
   updated after the draw to min(1, b (1/2 / f)^(1/N)), f the fraction of the
   drawn configurations with s = s' on every site (f = 0 counts as 1/4), so
   that repeated steps hold diagonal draws near half.  Strips run in FP64
   whatever desc->precision says.  A chain whose marginals at a site all
   vanish (or, with reweighting, whose only digits of nonzero marginal are
   diagonal while *b_diag = 0) records PEPS_ERR_ZERO_AMPLITUDE (non-finite
   marginals or b_diag PEPS_ERR_NONFINITE), gets log_p = -inf and zero
   digits from that site on.  For fermionic descs the
   draw is not restricted to even parity: a parity-even ansatz gives odd
   configurations zero weight by itself, and otherwise an odd draw gets
   importance weight 0.  ws: peps_direct_workspace_bytes(desc, n_chains,
   chi_dl).  The double-layer tensors and their bottom boundaries depend on
   theta only: with reuse_double_layer = 1 the call takes them from ws as
   the previous call on this workspace left them (same desc, chi_dl and
   theta, unchanged since, any number of chains; the caller guarantees it),
   with 0 it computes them. */
peps_status peps_direct_sample(const peps_desc* desc, const double* theta, int32_t n_chains, int32_t chi_dl,
                               uint64_t seed, uint64_t draw, int32_t reweight, double* b_diag, int32_t update_b,
                               int32_t reuse_double_layer, uint8_t* configs, double* log_p, int32_t* status,
                               void* ws, size_t ws_bytes, peps_trace* trace, peps_stream_t stream);

/* Importance weights of directly drawn samples (Eq. A7): weights[i] =
   exp(2 log_abs[i] - log_p[i] - m), m the largest finite value of
   2 log_abs - log_p, and 0 where log_abs or log_p is -inf.  The weights are
   scaled so that the largest is 1; pass them as `weights` to sr_cg_solve and
   peps_sample_stats.  n in [1, 2^30]. */
peps_status peps_importance_weights(int64_t n, const double* log_abs, const double* log_p, double* weights,
                                    peps_stream_t stream);

/* ---- instrumentation (not part of the method) --------------------------- */

/* Kernel classes of a trace. */
enum {
  PEPS_K_COMPRESS = 0, /* boundary row absorption + QR/SVD truncation       */
  PEPS_K_MOVES1 = 1,   /* Metropolis passes inside a row (one-row strips)   */
  PEPS_K_MOVES2 = 2,   /* vertical exchanges (two-row strips)               */
  PEPS_K_MEAS1 = 3,    /* O rows, in-row E_loc terms, log|psi|              */
  PEPS_K_MEAS2 = 4,    /* cross-row E_loc terms                             */
  PEPS_K_FINAL = 5,    /* per-sample outputs (and the FP64 re-evaluation of
                          ill-conditioned samples of the mixed path)        */
  PEPS_K_SR = 6,       /* all SR / CG kernels of one sr_cg_solve call       */
  PEPS_K_DIRECT = 7,   /* direct sampling: double layer, per-row draws      */
  PEPS_N_KCLASS = 8
};

/* Host: a trace with room for `capacity` timed launches (two HIP events
   each, created on the current device).  NULL if capacity < 1 or an event
   cannot be created.  Launches beyond the capacity are not timed. */
peps_trace* peps_trace_create(int32_t capacity);

/* Host: releases the events and the handle (NULL is a no-op). */
void peps_trace_destroy(peps_trace* trace);

/* Progress hook of a trace: fn(user, kernel_class, launch) is called once
   each timed launch of a call that receives the trace has completed (the
   library enqueues it after the launch's closing event with
   hipLaunchHostFunc on the call's stream; launch counts the trace's launches
   from 0 since its last read).  It runs on a HIP runtime thread, holds up
   later work of that stream while it runs, and must neither call HIP nor
   wait for anything the caller's thread may hold while it waits on the
   stream (an interpreter lock, say).  NULL fn removes the hook.
   PEPS_ERR_ARG for a NULL trace.  For long calls on large lattices, where
   one call can run for minutes. */
typedef void (*peps_progress_fn)(void* user, int32_t kernel_class, int32_t launch);
peps_status peps_trace_set_progress(peps_trace* trace, peps_progress_fn fn, void* user);

/* A ready-made hook: writes one line "[peps] <user> class <kernel_class>
   launch <launch> done (<t> s)" to stderr and flushes it (user: a
   NUL-terminated label, or NULL; t: seconds since the first line the
   process printed). */
void peps_progress_stderr(void* user, int32_t kernel_class, int32_t launch);

/* Host: synchronises the recorded events and adds, per kernel class, the
   summed duration in milliseconds to ms[PEPS_N_KCLASS] and the number of
   timed launches (one sr_cg_solve call counts as one) to
   launches[PEPS_N_KCLASS]; then empties the trace.  PEPS_ERR_ARG for a NULL
   trace, PEPS_ERR_HIP if an event query failed. */
peps_status peps_trace_read(peps_trace* trace, double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* PEPS_H */
