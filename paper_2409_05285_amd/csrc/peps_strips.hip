// Strip kernels (one workgroup per chain, at most 128 registers per lane so
// that four workgroups share a CU): Metropolis moves inside a row and
// between two rows, and the measurement of a configuration (log|psi|, local
// energy, O rows), all from one-row and two-row strips between fixed top and
// bottom boundary MPS.
//
// Each kernel is a template on the contraction type T.  T = double is the
// FP64 path.  T = float is the mixed-precision path: theta and the boundary
// tensors are read from FP32 copies, every strip contraction runs on FP32
// MFMA with FP32 accumulation, and each environment is stored scaled by an
// exact power of two chosen from its largest element (the exponents are
// carried in integers).  Ratios, log-amplitudes, energies and O entries are
// formed in FP64 from the FP32 contraction results and those exponents.
#include <math.h>

#include <type_traits>

#include "peps_chain.hpp"
#include "peps_kernels.hpp"

namespace peps {

namespace {

constexpr int NWAVE = NT / 64;

// Exponent bookkeeping of one stored environment: the true tensor is the
// stored one times 2^E, and the largest stored magnitude lies in
// [0.5, 1) * 2^s (s = 0 for an environment that is not tracked).  A step
// that consumes it scales its own output by 2^-s, so that output carries
// E + s.
struct Env {
  int E, s;
};

template <typename T> struct Prec;
template <> struct Prec<double> {
  __device__ static inline double scale(int) { return 1.0; }
  __device__ static inline float* track(float*) { return nullptr; }
  __device__ static inline int shift(const float*) { return 0; }
};
template <> struct Prec<float> {
  // 2^-s as an exact FP32 value (s clamped to the normal range)
  __device__ static inline float scale(int s) { return ldexpf(1.0f, -s); }
  __device__ static inline float* track(float* wmax) { return wmax; }
  __device__ static inline int shift(const float* wmax) {
    float m = 0.0f;
    for (int w = 0; w < NWAVE; ++w) m = fmaxf(m, wmax[w]);
    if (!(m > 0.0f) || !isfinite(m)) return 0;
    int e;
    frexpf(m, &e);
    return e < -125 ? -125 : (e > 125 ? 125 : e);
  }
};

// Output exponent of a step whose input carried `in` (applied scale 2^-in.s).
__device__ inline Env next_env(Env in, int s_out) { return Env{in.E + in.s, s_out}; }

// Ratio x / y of two tracked scalars, in FP64.
__device__ inline double tracked_ratio(double xm, int xE, double ym, int yE) { return ldexp(xm / ym, xE - yE); }

// Shared state of a strip kernel.
template <typename T>
struct StripShared {
  Geo geo;
  double red[NT];
  StripCtx<T> sc;
  uint8_t S[MAX_SITES];
  T one;
  float wmax[NWAVE];
  int Re[MAX_L + 1];   // exponents of the right environments
  int Rs[MAX_L + 1];
  int odd;             // fermionic tensors: the configuration has odd total parity
};

template <typename T>
__device__ inline void strip_prologue(const Prob& P, StripShared<T>& sh, const uint8_t* cfg) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    build_geo(P, sh.geo);
    sh.one = T(1);
  }
  for (int i = tid; i < P.N; i += NT) sh.S[i] = (uint8_t)digit_at(P, cfg, i);
  __syncthreads();
  if (P.fermionic) {
    // Z2-graded parity-even tensors: an odd total parity means rho = 0
    // exactly, decided here in integer arithmetic
    if (tid == 0) {
      int par = 0;
      for (int i = 0; i < P.N; ++i) par ^= digit_parity(P, sh.S[i]);
      sh.odd = par;
    }
    __syncthreads();
  } else if (tid == 0) {
    sh.odd = 0;
  }
}

// Error bookkeeping of the FP32 strips (mixed precision).  The strip
// amplitude rho is formed once from the right environments; the left pass
// forms it again at every column cut c as <L_c, R_{c+1}>, in a different
// rounding order.  The largest |rho_c / rho - 1| over the cuts samples the
// rounding error of rho and of the environments (dev), and u32 times the
// cancellation sum|L_c R_{c+1}| / |sum L_c R_{c+1}| of those dots bounds
// the last step's share (kap).  Each local-energy term coef rho(S') / rho
// adds its magnitude to `a`.  The three values go to the chain's record;
// k_redo_flags turns them into an error estimate.
constexpr double U32 = 0x1.0p-24;

struct ErrAcc {
  double dev = 0.0, kap = 0.0, a = 0.0;
};

__device__ inline void err_store(double* dst, const ErrAcc& ea) {
  dst[0] = ea.dev;
  dst[1] = ea.kap;
  dst[2] = ea.a;
}

// sum x_i y_i and sum |x_i y_i| (in FP64), identical on every thread.
template <typename T>
__device__ inline void wg_dot_abs(const T* x, const T* y, int n, double* red, double& dot, double& adot) {
  double s = 0.0, a = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) {
    const double p = (double)x[i] * (double)y[i];
    s += p;
    a += fabs(p);
  }
  dot = wg_sum(s, red);
  adot = wg_sum(a, red);
}

__device__ inline void err_cut(ErrAcc& ea, double d, double ad, int dE, double rho, int rhoE) {
  const double q = tracked_ratio(d, dE, rho, rhoE);
  ea.dev = fmax(ea.dev, fabs(q - 1.0));
  ea.kap = fmax(ea.kap, d != 0.0 ? U32 * ad / fabs(d) : INFINITY);
}

__device__ inline void err_term(ErrAcc& ea, double term) { ea.a += fabs(term); }

// Scratch tensors of a strip kernel inside the chain workspace.
template <typename T>
struct StripBufs {
  T *R, *Lb0, *Lb1, *tA, *tB, *X0, *X1;
};

template <typename T>
__device__ inline StripBufs<T> strip_bufs(const Prob& P, const ChainWS& w) {
  StripBufs<T> b;
  b.R = (T*)w.R;
  T* L = (T*)w.L;
  b.Lb0 = L;
  b.Lb1 = L + P.ES;
  b.tA = L + 2 * (size_t)P.ES;
  b.tB = L + 3 * (size_t)P.ES;
  b.X0 = (T*)w.X;
  b.X1 = b.X0 + P.XS;
  return b;
}

// One-row environments from the right: R_c (c = L2..0) at R + c*ES.
template <typename T>
__device__ inline void right_envs1(const Prob& P, StripShared<T>& sh, const T* theta, const StripBufs<T>& b, int r) {
  using PR = Prec<T>;
  if (threadIdx.x == 0) {
    b.R[(size_t)P.L2 * P.ES] = T(1);
    sh.Re[P.L2] = 0;
    sh.Rs[P.L2] = 0;
  }
  __syncthreads();
  Env e{0, 0};
  for (int c = P.L2 - 1; c >= 0; --c) {
    const int i = r * P.L2 + c;
    rstep1<T>(b.R + (size_t)c * P.ES, b.R + (size_t)(c + 1) * P.ES, sh.sc.T_[c], sh.sc.tD[c],
              slice_ptr(P, sh.geo, theta, r, c, sh.S[i]), wdim(P, r, c), sh.sc.B[c], sh.sc.bD[c], b.X0, b.X1,
              PR::scale(e.s), PR::track(sh.wmax));
    e = next_env(e, PR::shift(sh.wmax));
    if (threadIdx.x == 0) {
      sh.Re[c] = e.E;
      sh.Rs[c] = e.s;
    }
  }
  __syncthreads();
}

template <typename T>
__device__ inline void right_envs2(const Prob& P, StripShared<T>& sh, const T* theta, const StripBufs<T>& b, int r) {
  using PR = Prec<T>;
  if (threadIdx.x == 0) {
    b.R[(size_t)P.L2 * P.ES] = T(1);
    sh.Re[P.L2] = 0;
    sh.Rs[P.L2] = 0;
  }
  __syncthreads();
  Env e{0, 0};
  for (int c = P.L2 - 1; c >= 0; --c) {
    const int i = r * P.L2 + c, j = (r + 1) * P.L2 + c;
    rstep2<T>(b.R + (size_t)c * P.ES, b.R + (size_t)(c + 1) * P.ES, sh.sc.T_[c], sh.sc.tD[c],
              slice_ptr(P, sh.geo, theta, r, c, sh.S[i]), wdim(P, r, c),
              slice_ptr(P, sh.geo, theta, r + 1, c, sh.S[j]), wdim(P, r + 1, c), sh.sc.B[c], sh.sc.bD[c], b.X0,
              b.X1, PR::scale(e.s), PR::track(sh.wmax));
    e = next_env(e, PR::shift(sh.wmax));
    if (threadIdx.x == 0) {
      sh.Re[c] = e.E;
      sh.Rs[c] = e.s;
    }
  }
  __syncthreads();
}

template <typename T>
__device__ inline int env1_size(const Prob& P, const StripCtx<T>& sc, int r, int c) {
  return sc.tD[c].n2 * wdim(P, r, c).n2 * sc.bD[c].n2;
}

template <typename T>
__device__ inline int env2_size(const Prob& P, const StripCtx<T>& sc, int r, int c) {
  return sc.tD[c].n2 * wdim(P, r, c).n2 * wdim(P, r + 1, c).n2 * sc.bD[c].n2;
}

// One column of the one-row strip from the left, with exponent tracking.
template <typename T>
__device__ inline Env lstep1_t(const Prob& P, StripShared<T>& sh, const StripBufs<T>& b, T* out, const T* L, Env eL,
                               const T* theta, int r, int c, int Sc) {
  using PR = Prec<T>;
  lstep1<T>(out, L, sh.sc.T_[c], sh.sc.tD[c], slice_ptr(P, sh.geo, theta, r, c, Sc), wdim(P, r, c), sh.sc.B[c],
            sh.sc.bD[c], b.X0, b.X1, PR::scale(eL.s), PR::track(sh.wmax));
  return next_env(eL, PR::shift(sh.wmax));
}

// One column of the two-row strip from the left, with exponent tracking.
template <typename T>
__device__ inline Env lstep2_t(const Prob& P, StripShared<T>& sh, const StripBufs<T>& b, T* out, const T* L, Env eL,
                               const T* theta, int r, int c, int S1, int S2) {
  using PR = Prec<T>;
  lstep2<T>(out, L, sh.sc.T_[c], sh.sc.tD[c], slice_ptr(P, sh.geo, theta, r, c, S1), wdim(P, r, c),
            slice_ptr(P, sh.geo, theta, r + 1, c, S2), wdim(P, r + 1, c), sh.sc.B[c], sh.sc.bD[c], b.X0, b.X1,
            PR::scale(eL.s), PR::track(sh.wmax));
  return next_env(eL, PR::shift(sh.wmax));
}

}  // namespace

// ---------------------------------------------------------------------------
// Metropolis passes inside row r: horizontal exchanges, then site moves.
template <typename T>
__global__ void __launch_bounds__(NT, 4) k_moves1(Prob P, int r, const T* __restrict__ theta, uint8_t* configs,
                                               uint64_t seed, uint64_t gsweep0, const uint64_t* gctr, double* ws,
                                               int32_t* n_accept, int32_t* status) {
  // global sweep index: the host's base plus the device counter, if any
  const uint64_t gsweep = gsweep0 + (gctr ? gctr[0] : 0ull);
  __shared__ StripShared<T> sh;
  const int tid = threadIdx.x;
  const int ch = blockIdx.x;
  ChainWS w = chain_ws(P, ws, ch);
  uint8_t* cfg = configs + (size_t)ch * P.N;
  strip_prologue(P, sh, cfg);
  build_strip<T>(P, sh.geo, w, r, r + 1, &sh.one, sh.sc);
  __syncthreads();
  if (sh.odd) {   // fermionic tensors, odd total parity: rho = 0, the chain cannot move
    set_status(status, PEPS_ERR_ZERO_AMPLITUDE);
    return;
  }
  const StripBufs<T> b = strip_bufs<T>(P, w);
  uint8_t* S = sh.S;
  T* Lb[2] = {b.Lb0, b.Lb1};
  int acc_h = 0, acc_s = 0;
  int slot = slot_base(P, r);

  // horizontal exchanges
  right_envs1(P, sh, theta, b, r);
  double rho = (double)b.R[0];
  int rhoE = sh.Re[0];
  const T* Lc = &sh.one;
  Env eL{0, 0};
  int cur = 0;
  for (int c = 0; c < P.L2 - 1; ++c) {
    const int i = r * P.L2 + c, j = i + 1;
    for (int k = 0; k < P.nb_moves; ++k, ++slot) {
      int ni, nj;
      if (!bond_proposal(P, S[i], S[j], k, ni, nj)) continue;
      const Env eA = lstep1_t(P, sh, b, b.tA, Lc, eL, theta, r, c, ni);
      const Env eB = lstep1_t(P, sh, b, b.tB, b.tA, eA, theta, r, c + 1, nj);
      const double rn = wg_dot<T>(b.tB, b.R + (size_t)(c + 2) * P.ES, env1_size(P, sh.sc, r, c + 1), sh.red);
      const int rnE = eB.E + sh.Re[c + 2];
      bool acc = false;
      if (rho == 0.0) {
        set_status(status, PEPS_ERR_ZERO_AMPLITUDE);
      } else {
        const double R = tracked_ratio(rn, rnE, rho, rhoE);
        if (!isfinite(R)) set_status(status, PEPS_ERR_NONFINITE);
        acc = metropolis(P, R, slot_uniform(seed, ch, gsweep, slot));
      }
      if (acc) {
        if (tid == 0) { S[i] = (uint8_t)ni; S[j] = (uint8_t)nj; }
        rho = rn;
        rhoE = rnE;
        ++acc_h;
      }
      __syncthreads();
    }
    eL = lstep1_t(P, sh, b, Lb[cur], Lc, eL, theta, r, c, S[i]);
    Lc = Lb[cur];
    cur ^= 1;
  }

  // site moves
  right_envs1(P, sh, theta, b, r);
  rho = (double)b.R[0];
  rhoE = sh.Re[0];
  Lc = &sh.one;
  eL = Env{0, 0};
  for (int c = 0; c < P.L2; ++c) {
    const int i = r * P.L2 + c;
    for (int k = 0; k < P.ns_moves; ++k, ++slot) {
      int ni;
      if (!site_proposal(P, S[i], k, ni)) continue;
      const Env eA = lstep1_t(P, sh, b, b.tA, Lc, eL, theta, r, c, ni);
      const double rn = wg_dot<T>(b.tA, b.R + (size_t)(c + 1) * P.ES, env1_size(P, sh.sc, r, c), sh.red);
      const int rnE = eA.E + sh.Re[c + 1];
      bool acc = false;
      if (rho == 0.0) {
        set_status(status, PEPS_ERR_ZERO_AMPLITUDE);
      } else {
        const double R = tracked_ratio(rn, rnE, rho, rhoE);
        if (!isfinite(R)) set_status(status, PEPS_ERR_NONFINITE);
        acc = metropolis(P, R, slot_uniform(seed, ch, gsweep, slot));
      }
      if (acc) {
        if (tid == 0) S[i] = (uint8_t)ni;
        rho = rn;
        rhoE = rnE;
        ++acc_s;
      }
      __syncthreads();
    }
    if (c < P.L2 - 1) {
      eL = lstep1_t(P, sh, b, Lb[cur], Lc, eL, theta, r, c, S[i]);
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
template <typename T>
__global__ void __launch_bounds__(NT, 4) k_moves2(Prob P, int r, const T* __restrict__ theta, uint8_t* configs,
                                               uint64_t seed, uint64_t gsweep0, const uint64_t* gctr, double* ws,
                                               int32_t* n_accept, int32_t* status) {
  // global sweep index: the host's base plus the device counter, if any
  const uint64_t gsweep = gsweep0 + (gctr ? gctr[0] : 0ull);
  __shared__ StripShared<T> sh;
  const int tid = threadIdx.x;
  const int ch = blockIdx.x;
  ChainWS w = chain_ws(P, ws, ch);
  uint8_t* cfg = configs + (size_t)ch * P.N;
  strip_prologue(P, sh, cfg);
  build_strip<T>(P, sh.geo, w, r, r + 2, &sh.one, sh.sc);
  __syncthreads();
  if (sh.odd) {   // fermionic tensors, odd total parity: rho = 0, the chain cannot move
    set_status(status, PEPS_ERR_ZERO_AMPLITUDE);
    return;
  }
  const StripBufs<T> b = strip_bufs<T>(P, w);
  uint8_t* S = sh.S;
  T* Lb[2] = {b.Lb0, b.Lb1};
  int acc_v = 0;
  int slot = slot_base(P, r) + P.nb_moves * (P.L2 - 1) + P.ns_moves * P.L2;
  right_envs2(P, sh, theta, b, r);
  double rho = (double)b.R[0];
  int rhoE = sh.Re[0];
  const T* Lc = &sh.one;
  Env eL{0, 0};
  int cur = 0;
  for (int c = 0; c < P.L2; ++c) {
    const int i = r * P.L2 + c, j = (r + 1) * P.L2 + c;
    for (int k = 0; k < P.nb_moves; ++k, ++slot) {
      int ni, nj;
      if (!bond_proposal(P, S[i], S[j], k, ni, nj)) continue;
      const Env eA = lstep2_t(P, sh, b, b.tA, Lc, eL, theta, r, c, ni, nj);
      const double rn = wg_dot<T>(b.tA, b.R + (size_t)(c + 1) * P.ES, env2_size(P, sh.sc, r, c), sh.red);
      const int rnE = eA.E + sh.Re[c + 1];
      bool acc = false;
      if (rho == 0.0) {
        set_status(status, PEPS_ERR_ZERO_AMPLITUDE);
      } else {
        const double R = tracked_ratio(rn, rnE, rho, rhoE);
        if (!isfinite(R)) set_status(status, PEPS_ERR_NONFINITE);
        acc = metropolis(P, R, slot_uniform(seed, ch, gsweep, slot));
      }
      if (acc) {
        if (tid == 0) { S[i] = (uint8_t)ni; S[j] = (uint8_t)nj; }
        rho = rn;
        rhoE = rnE;
        ++acc_v;
      }
      __syncthreads();
    }
    if (c < P.L2 - 1) {
      eL = lstep2_t(P, sh, b, Lb[cur], Lc, eL, theta, r, c, S[i], S[j]);
      Lc = Lb[cur];
      cur ^= 1;
    }
  }
  for (int i = tid; i < P.N; i += NT) cfg[i] = S[i];
  if (tid == 0 && n_accept) n_accept[(size_t)ch * PEPS_N_MOVE_TYPES + 2] += acc_v;
}

// ---------------------------------------------------------------------------
// Measurement of row r (one-row strip): the O blocks of the row's sites, the
// local-energy terms inside the row (exchanges, or hops with their
// Jordan-Wigner signs), and (last row) log|psi| and its sign.
// epart layout per chain: [0, L1) in-row terms, [L1, 2 L1) cross-row terms,
// [2 L1] log|psi|, [2 L1 + 1] sign.
// One row of the measurement of chain ch, whose boundaries and record are in
// w; b is the scratch of the calling workgroup.
template <typename T>
__device__ void meas1_row(const Prob& P, StripShared<T>& sh, const ChainWS& w, const StripBufs<T>& b, int r,
                          int ch, const T* __restrict__ theta, const uint8_t* configs, double* O_rows, int want_e,
                          int32_t* status) {
  using PR = Prec<T>;
  constexpr bool kErr = std::is_same<T, float>::value;
  const int tid = threadIdx.x;
  strip_prologue(P, sh, configs + (size_t)ch * P.N);
  build_strip<T>(P, sh.geo, w, r, r + 1, &sh.one, sh.sc);
  __syncthreads();
  const uint8_t* S = sh.S;
  T* Lb[2] = {b.Lb0, b.Lb1};
  double rho = 0.0;
  int rhoE = 0;
  if (!sh.odd) {
    right_envs1(P, sh, theta, b, r);
    rho = (double)b.R[0];
    rhoE = sh.Re[0];
  }
  if (rho == 0.0 || !isfinite(rho)) {
    // a zero amplitude has log|psi| = -inf (sign 0); its local energy and O
    // row are undefined
    set_status(status, rho == 0.0 ? PEPS_ERR_ZERO_AMPLITUDE : PEPS_ERR_NONFINITE);
    if (tid == 0) {
      w.epart[r] = NAN;
      if (r == P.L1 - 1) { w.epart[2 * P.L1] = rho == 0.0 ? -INFINITY : NAN; w.epart[2 * P.L1 + 1] = 0.0; }
      if (kErr) w.epart[epart_err1(P) + 3 * r] = NAN;
    }
    return;
  }
  if (r == P.L1 - 1 && tid == 0) {
    const double ls = r >= 1 ? w.lstop[r - 1] : 0.0;
    w.epart[2 * P.L1] = ls + log(fabs(rho)) + (double)rhoE * M_LN2;
    w.epart[2 * P.L1 + 1] = rho > 0.0 ? 1.0 : -1.0;
  }
  double e = 0.0;
  ErrAcc ea;
  double* Orow = O_rows ? O_rows + (size_t)ch * P.nnz : nullptr;
  const double inv = 1.0 / rho;
  const T* Lc = &sh.one;
  Env eL{0, 0};
  int cur = 0;
  for (int c = 0; c < P.L2; ++c) {
    const int i = r * P.L2 + c;
    const Dim4 wd = wdim(P, r, c);
    if (Orow) {
      // env * 2^(eL.E + eL.s + E_R + s_R) is the true site environment; the
      // stored one carries the scale 2^-(eL.s + s_R).
      site_env1<T>(b.tA, Lc, sh.sc.T_[c], sh.sc.tD[c], sh.sc.B[c], sh.sc.bD[c], b.R + (size_t)(c + 1) * P.ES, wd.n0,
                   wd.n2, b.X0, b.X1, PR::scale(eL.s + sh.Rs[c + 1]));
      const double f = ldexp(inv, eL.E + eL.s + sh.Re[c + 1] + sh.Rs[c + 1] - rhoE);
      const int bs = wd.n0 * wd.n1 * wd.n2 * wd.n3;
      for (int q = tid; q < bs; q += NT) Orow[sh.geo.ooff[i] + q] = (double)b.tA[q] * f;
      __syncthreads();
    }
    if (want_e && c < P.L2 - 1) {
      for (int k = 0; k < P.nb_moves; ++k) {
        int ni, nj;
        if (!bond_proposal(P, S[i], S[i + 1], k, ni, nj)) continue;
        const Env eA = lstep1_t(P, sh, b, b.tA, Lc, eL, theta, r, c, ni);
        const Env eB = lstep1_t(P, sh, b, b.tB, b.tA, eA, theta, r, c + 1, nj);
        const T* Rn = b.R + (size_t)(c + 2) * P.ES;
        const int nE = eB.E + sh.Re[c + 2];
        const double rn = wg_dot<T>(b.tB, Rn, env1_size(P, sh.sc, r, c + 1), sh.red);
        const double term = bond_coeff(P, S, i, i + 1, k, P.J1) * tracked_ratio(rn, nE, rho, rhoE);
        e += term;
        if (kErr) err_term(ea, term);
      }
    }
    if (c < P.L2 - 1) {
      eL = lstep1_t(P, sh, b, Lb[cur], Lc, eL, theta, r, c, S[i]);
      Lc = Lb[cur];
      cur ^= 1;
      if (kErr) {
        double d, ad;
        wg_dot_abs<T>(Lc, b.R + (size_t)(c + 1) * P.ES, env1_size(P, sh.sc, r, c), sh.red, d, ad);
        err_cut(ea, d, ad, eL.E + sh.Re[c + 1], rho, rhoE);
      }
    }
  }
  if (tid == 0) {
    w.epart[r] = e;
    if (kErr) err_store(w.epart + epart_err1(P) + 3 * r, ea);
  }
}

template <typename T>
__global__ void __launch_bounds__(NT, 4) k_meas1(Prob P, int r, const T* __restrict__ theta, const uint8_t* configs,
                                                 double* ws, double* O_rows, int want_e, int32_t* status) {
  __shared__ StripShared<T> sh;
  const int ch = blockIdx.x;
  const ChainWS w = chain_ws(P, ws, ch);
  meas1_row<T>(P, sh, w, strip_bufs<T>(P, w), r, ch, theta, configs, O_rows, want_e, status);
}

// Cross-row local-energy terms between rows r and r+1 (two-row strip):
// vertical bonds (exchanges, or hops with their Jordan-Wigner signs), and
// the spin exchange on next-nearest-neighbour bonds when J2 != 0.
template <typename T>
__device__ void meas2_row(const Prob& P, StripShared<T>& sh, const ChainWS& w, const StripBufs<T>& b, int r,
                          int ch, const T* __restrict__ theta, const uint8_t* configs, int32_t* status) {
  constexpr bool kErr = std::is_same<T, float>::value;
  const int tid = threadIdx.x;
  strip_prologue(P, sh, configs + (size_t)ch * P.N);
  build_strip<T>(P, sh.geo, w, r, r + 2, &sh.one, sh.sc);
  __syncthreads();
  const uint8_t* S = sh.S;
  T* Lb[2] = {b.Lb0, b.Lb1};
  double rho = 0.0;
  int rhoE = 0;
  if (!sh.odd) {
    right_envs2(P, sh, theta, b, r);
    rho = (double)b.R[0];
    rhoE = sh.Re[0];
  }
  if (rho == 0.0 || !isfinite(rho)) {
    set_status(status, rho == 0.0 ? PEPS_ERR_ZERO_AMPLITUDE : PEPS_ERR_NONFINITE);
    if (tid == 0) {
      w.epart[P.L1 + r] = NAN;
      if (kErr) w.epart[epart_err2(P) + 3 * r] = NAN;
    }
    return;
  }
  double e = 0.0;
  ErrAcc ea;
  // one local-energy term coef * rho(S') / rho from the environment tX of
  // the modified columns and the right environment Rn
  auto term = [&](double coef, const T* tX, const T* Rn, int n, int nE) {
    const double t = coef * tracked_ratio(wg_dot<T>(tX, Rn, n, sh.red), nE, rho, rhoE);
    e += t;
    if (kErr) err_term(ea, t);
  };
  const T* Lc = &sh.one;
  Env eL{0, 0};
  int cur = 0;
  for (int c = 0; c < P.L2; ++c) {
    const int i = r * P.L2 + c, j = (r + 1) * P.L2 + c;
    for (int k = 0; k < P.nb_moves; ++k) {
      int ni, nj;
      if (!bond_proposal(P, S[i], S[j], k, ni, nj)) continue;
      const Env eA = lstep2_t(P, sh, b, b.tA, Lc, eL, theta, r, c, ni, nj);
      term(bond_coeff(P, S, i, j, k, P.J1), b.tA, b.R + (size_t)(c + 1) * P.ES, env2_size(P, sh.sc, r, c),
           eA.E + sh.Re[c + 1]);
    }
    if (P.J2 != 0.0 && c < P.L2 - 1) {
      // spin exchange on the bonds (r,c)-(r+1,c+1) and (r,c+1)-(r+1,c), ket
      // then bra side (the J2 coupling of either model)
      for (int orient = 0; orient < 2; ++orient) {
        const int sa = orient == 0 ? i : i + 1;    // site in row r
        const int sbs = orient == 0 ? j + 1 : j;   // site in row r+1
        for (int side = 0; side < 2; ++side) {
          int na, nb;
          if (!spin_exchange(P, S[sa], S[sbs], side, na, nb)) continue;
          int s1c = S[i], s1n = S[i + 1], s2c = S[j], s2n = S[j + 1];
          if (orient == 0) { s1c = na; s2n = nb; } else { s1n = na; s2c = nb; }
          const Env eA = lstep2_t(P, sh, b, b.tA, Lc, eL, theta, r, c, s1c, s2c);
          const Env eB = lstep2_t(P, sh, b, b.tB, b.tA, eA, theta, r, c + 1, s1n, s2n);
          term(0.5 * P.J2, b.tB, b.R + (size_t)(c + 2) * P.ES, env2_size(P, sh.sc, r, c + 1), eB.E + sh.Re[c + 2]);
        }
      }
    }
    if (c < P.L2 - 1) {
      eL = lstep2_t(P, sh, b, Lb[cur], Lc, eL, theta, r, c, S[i], S[j]);
      Lc = Lb[cur];
      cur ^= 1;
      if (kErr) {
        double d, ad;
        wg_dot_abs<T>(Lc, b.R + (size_t)(c + 1) * P.ES, env2_size(P, sh.sc, r, c), sh.red, d, ad);
        err_cut(ea, d, ad, eL.E + sh.Re[c + 1], rho, rhoE);
      }
    }
  }
  if (tid == 0) {
    w.epart[P.L1 + r] = e;
    if (kErr) err_store(w.epart + epart_err2(P) + 3 * r, ea);
  }
}

template <typename T>
__global__ void __launch_bounds__(NT, 4) k_meas2(Prob P, int r, const T* __restrict__ theta, const uint8_t* configs,
                                                 double* ws, int32_t* status) {
  __shared__ StripShared<T> sh;
  const int ch = blockIdx.x;
  const ChainWS w = chain_ws(P, ws, ch);
  meas2_row<T>(P, sh, w, strip_bufs<T>(P, w), r, ch, theta, configs, status);
}

// Mixed precision: the FP64 measurement of the row strips k_redo_flags
// listed (list[0] = count, then items chain * 64 + kind, kind r < L1 the
// one-row strip r, L1 + r the two-row strip r).  The workgroups of the grid
// take the items round-robin, so that a few listed strips cost a few strip
// latencies instead of one launch per strip.  Workgroup g uses chain g's
// strip scratch (the grid has at most n workgroups).  A one-row strip whose
// amplitude estimate was above the bar also rewrites its O rows.
__global__ void __launch_bounds__(NT, 4) k_remeasure(Prob P, const double* __restrict__ theta,
                                                     const uint8_t* configs, double* ws, const int32_t* list,
                                                     double* O_rows, int want_e, int32_t* status) {
  __shared__ StripShared<double> sh;
  const int64_t items = list[0];
  const StripBufs<double> b = strip_bufs<double>(P, chain_ws(P, ws, blockIdx.x));
  for (int64_t j = blockIdx.x; j < items; j += gridDim.x) {
    const int item = list[1 + j];
    const int ch = item >> 6, kind = item & 63;
    const ChainWS w = chain_ws(P, ws, ch);
    const bool with_O = ((((uint32_t)w.epart[epart_mask(P)]) >> kind) & 1u) != 0;
    if (kind < P.L1)
      meas1_row<double>(P, sh, w, b, kind, ch, theta, configs, with_O ? O_rows : nullptr, want_e, status);
    else
      meas2_row<double>(P, sh, w, b, kind - P.L1, ch, theta, configs, status);
    __syncthreads();
  }
}

// FP32 copy of theta for the mixed-precision strips.
__global__ void k_theta32(const double* __restrict__ theta, float* __restrict__ t32, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    t32[i] = (float)theta[i];
}

// Device sweep counter: advanced once per call, after every kernel of the
// call has read it (stream order), so graph replays draw fresh numbers.
__global__ void k_advance_counter(uint64_t* ctr, uint64_t n) {
  if (threadIdx.x == 0) ctr[0] = ctr[0] + n;
}

__global__ void k_copy_bytes(uint8_t* __restrict__ dst, const uint8_t* __restrict__ src, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t n16 = ((uintptr_t)dst % 16 == 0 && (uintptr_t)src % 16 == 0) ? n / 16 : 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
  for (int64_t i = n16 * 16 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
hipError_t launch_copy_bytes(uint8_t* dst, const uint8_t* src, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n / 16 + 255) / 256;
  hipLaunchKernelGGL(k_copy_bytes, dim3(blocks < 1 ? 1 : (blocks > 1024 ? 1024 : (int)blocks)), dim3(256), 0, st,
                     dst, src, n);
  return hipGetLastError();
}

hipError_t launch_advance_counter(uint64_t* ctr, uint64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_advance_counter, dim3(1), dim3(64), 0, st, ctr, n);
  return hipGetLastError();
}

hipError_t launch_theta32(const Prob& P, const double* theta, float* t32, hipStream_t st) {
  const int blocks = (int)((P.np + 255) / 256 < 1024 ? (P.np + 255) / 256 : 1024);
  hipLaunchKernelGGL(k_theta32, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, theta, t32, P.np);
  return hipGetLastError();
}

hipError_t launch_moves1(const Prob& P, int n, int r, const double* theta, const float* t32, uint8_t* configs,
                         uint64_t seed, uint64_t gsweep, const uint64_t* gctr, double* ws, int32_t* n_accept,
                         int32_t* status, hipStream_t st) {
  if (P.mixed)
    hipLaunchKernelGGL(k_moves1<float>, dim3(n), dim3(NT), 0, st, P, r, t32, configs, seed, gsweep, gctr, ws, n_accept,
                       status);
  else
    hipLaunchKernelGGL(k_moves1<double>, dim3(n), dim3(NT), 0, st, P, r, theta, configs, seed, gsweep, gctr, ws, n_accept,
                       status);
  return hipGetLastError();
}

hipError_t launch_moves2(const Prob& P, int n, int r, const double* theta, const float* t32, uint8_t* configs,
                         uint64_t seed, uint64_t gsweep, const uint64_t* gctr, double* ws, int32_t* n_accept,
                         int32_t* status, hipStream_t st) {
  if (P.mixed)
    hipLaunchKernelGGL(k_moves2<float>, dim3(n), dim3(NT), 0, st, P, r, t32, configs, seed, gsweep, gctr, ws, n_accept,
                       status);
  else
    hipLaunchKernelGGL(k_moves2<double>, dim3(n), dim3(NT), 0, st, P, r, theta, configs, seed, gsweep, gctr, ws, n_accept,
                       status);
  return hipGetLastError();
}

hipError_t launch_meas1(const Prob& P, int n, int r, const double* theta, const float* t32, const uint8_t* configs,
                        double* ws, double* O_rows, int want_e, int32_t* status, hipStream_t st) {
  if (P.mixed)
    hipLaunchKernelGGL(k_meas1<float>, dim3(n), dim3(NT), 0, st, P, r, t32, configs, ws, O_rows, want_e, status);
  else
    hipLaunchKernelGGL(k_meas1<double>, dim3(n), dim3(NT), 0, st, P, r, theta, configs, ws, O_rows, want_e, status);
  return hipGetLastError();
}

hipError_t launch_meas2(const Prob& P, int n, int r, const double* theta, const float* t32, const uint8_t* configs,
                        double* ws, int32_t* status, hipStream_t st) {
  if (P.mixed)
    hipLaunchKernelGGL(k_meas2<float>, dim3(n), dim3(NT), 0, st, P, r, t32, configs, ws, status);
  else
    hipLaunchKernelGGL(k_meas2<double>, dim3(n), dim3(NT), 0, st, P, r, theta, configs, ws, status);
  return hipGetLastError();
}

hipError_t launch_remeasure(const Prob& P, int n, const double* theta, const uint8_t* configs, double* ws,
                            const int32_t* list, double* O_rows, int want_e, int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_remeasure, dim3(n), dim3(NT), 0, st, P, theta, configs, ws, list, O_rows, want_e, status);
  return hipGetLastError();
}

}  // namespace peps
