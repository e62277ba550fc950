// rk_device.hpp -- RKCK / RKC drivers for one ODE system per lane, and the
// kernels that schedule them.
//
// Method: Niemeyer & Sung (2014).  RKCK: Table 1, Sec. 2.1 stage equations,
// error estimate and step-size rule, Sec. 3.1 driver.  RKC: Sec. 2.2 stage
// recursion, coefficients, error estimate and RMS norm, step-size rules,
// initial step and stage count, Sec. 3.2 driver; Appendix nonlinear power
// method.  Readings where the paper is silent or garbled:
//   * eps = rtol, delta = atol / rtol (TINY when atol = 0) in the RKCK scale;
//   * P1 = 0.1; RKCK keeps f(t, y) across a rejection;
//   * RKC: b_0 = b_1 = b_2; power-method convergence |sigma_k - sigma_{k-1}|
//     <= 0.01 max(sigma_k, 1/hMax); restart state (no memory across calls,
//     v = f(t0, y0)); a non-finite RKC error is a rejection with h *= P1;
//     rejection step 0.8 h / err^(1/3) without a floor;
//   * guards: h below hMin after a rejection, a non-finite accepted state or
//     max_steps attempts end the system with a status code;
//   * exp, log and pow round a double-double evaluation (crmath.hpp): the
//     correctly rounded value but for ~2^-35 of calls.
// Every expression is written in the order of the reference evaluation and the
// library is built without contraction, so results are reproducible bit for bit.
//
// A problem type Prob supplies
//   static constexpr int N;             unknowns
//   static constexpr bool kColumns;     vectors in slot columns (else registers)
//   static constexpr int kLaneDoubles;  per-system constants kept in the slot
//   using Params;                       uniform data passed by value
//   struct Lane;                        per-system constants kept in registers
//   static void init(Lane&, const Params&, const double* g, int64_t i, int64_t n,
//                    double* slot);     slot[j * kLdsStride], j < kLaneDoubles
//   template <class VI, class VO>
//   static void rhs(const Lane&, const Params&, const VI& y, VO& f);
// Every right-hand side here is autonomous, so stage times are not formed.
//
// The slot of a lane is a set of columns with stride kLdsStride (the lanes of
// a wave interleaved, so a wave's access to one element is one contiguous
// 512-byte row): first the problem's kLaneDoubles constants, then vectors of
// N doubles.  Small systems keep their vectors in registers and their slot in
// LDS; large ones (kColumns) keep every vector in slot columns in a device
// workspace, with the right-hand side outlined as one function.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "crmath.hpp"
#include "rk_types.hpp"

namespace rkmi {

constexpr double kUround = 2.22e-16;
constexpr double kSafety = 0.9;
constexpr double kPGrow = -0.2;      // err^kPGrow: crm::pow_minus_fifth
constexpr double kPShrink = -0.25;   // err^kPShrink: crm::pow_minus_quarter
constexpr double kErrCon = 1.89e-4;
constexpr double kP1 = 0.1;
constexpr double kRkckHmin = 1.0e-20;

// Lanes per workgroup of every integration kernel (one wave64), which is also
// the stride of the per-lane columns in LDS.
constexpr int kLdsStride = 64;

enum : int32_t { kSysOk = 0, kSysNonFinite = 1, kSysHmin = 2, kSysMaxSteps = 3 };
enum : int { kStAccept = 0, kStReject, kStRhs, kStSrCalls, kStPowIters, kStMaxStages, kNStats };

// Read-only, wave-uniform data (the network constants of a launch).  On the
// device it is read through the constant address space, so the compiler can
// use scalar loads into scalar registers instead of holding the values in
// vector registers; the host build reads it plainly.
RKMI_HD double ld_uniform(const double* p, int k) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const __attribute__((address_space(4))) double*)p)[k];
#else
  return p[k];
#endif
}

// Zero, as a value the optimizer cannot see through: memory read at an offset
// that includes it stays where the source reads it (a loop-invariant read is
// not hoisted out of the integration loop into live registers).
RKMI_HD int opaque_zero() {
#if defined(__HIP_DEVICE_COMPILE__)
  int z = 0;
  asm volatile("" : "+s"(z));
  return z;
#else
  return 0;
#endif
}

// Waves per SIMD the integration kernels of a problem are compiled for: a
// problem may ask for more than the register allocator would choose by itself
// (Prob::kWavesPerEu), trading a few spilled bytes for latency hiding.
template <class P, class = void>
struct WavesPerEu {
  static constexpr int value = 1;
};
template <class P>
struct WavesPerEu<P, std::void_t<decltype(P::kWavesPerEu)>> {
  static constexpr int value = P::kWavesPerEu;
};

// Controller state carried from one call to the next instead of the restart
// (Sec. 3 mentions the alternative): rows of a [kCarryRows + N][n] array, the
// RKC eigenvector estimate in the last N rows; RKCK uses kCarryValid and
// kCarryH.  kCarryValid = 0 asks for the restart; a call leaves 1 when its
// system ended OK.  The carried next step is the one the controller wanted
// before the final step was cut to the interval end.
enum : int {
  kCarryValid = 0, kCarryH, kCarryHPrev, kCarryErrPrev, kCarrySigma, kCarryNstep,
  kCarryHavePrev, kCarryRows
};

// A vector of N unknowns held in registers.
template <int N>
struct RegVec {
  double a[N];
  RKMI_HD double& operator[](int k) { return a[k]; }
  RKMI_HD const double& operator[](int k) const { return a[k]; }
};

// A vector of N unknowns held in a slot column: element k at p[k * kLdsStride].
template <int N>
struct ColVec {
  double* p;
  RKMI_HD double& operator[](int k) const { return p[k * kLdsStride]; }
};

template <class Prob>
using Vec = typename std::conditional<Prob::kColumns, ColVec<Prob::N>, RegVec<Prob::N>>::type;

// Start of vector column `col` in a lane's slot.
template <class Prob>
RKMI_HD double* col_ptr(double* slot, int col) {
  return slot + (Prob::kLaneDoubles + col * Prob::N) * kLdsStride;
}

// A work vector: column `col` of the slot, or fresh registers.
template <class Prob>
RKMI_HD Vec<Prob> work_vec(double* slot, int col) {
  if constexpr (Prob::kColumns) {
    return ColVec<Prob::N>{col_ptr<Prob>(slot, col)};
  } else {
    (void)slot;
    (void)col;
    Vec<Prob> v;
    return v;
  }
}

// Column layouts of the two drivers (RKC's column 0, the power-method
// eigenvector, is also used by register-held systems).
enum : int { kCkY = 0, kCkF, kCkYt, kCkYe, kCkK1, kCkK2, kCkK3, kCkK4, kCkK5, kCkZ, kCkFs, kCkCols };
enum : int { kCV = 0, kCYn, kCFn, kCY, kCF1, kCWm2, kCFs, kCFv, kCCols };

// Doubles per lane of the slot a kernel needs.
template <class Prob, int Method>
constexpr int slot_doubles() {
  return Prob::kColumns ? Prob::kLaneDoubles + Prob::N * (Method == kMethodRkck ? kCkCols : kCCols)
                        : Prob::kLaneDoubles + (Method == kMethodRkc ? Prob::N : 0);
}

// The right-hand side over slot columns as one outlined function, so its code
// is not repeated at every call site.
template <class Prob>
__attribute__((noinline)) RKMI_HD void rhs_outlined(typename Prob::Lane L,
                                                    typename Prob::Params prm, double* y,
                                                    double* f) {
  const ColVec<Prob::N> yv{y};
  ColVec<Prob::N> fv{f};
  Prob::rhs(L, prm, yv, fv);
}

template <class Prob, class VI, class VO>
RKMI_HD void eval_rhs(const typename Prob::Lane& L, const typename Prob::Params& prm, const VI& y,
                      VO& f) {
  if constexpr (Prob::kColumns)
    rhs_outlined<Prob>(L, prm, y.p, f.p);
  else
    Prob::rhs(L, prm, y, f);
}

// Loops over the unknowns are unrolled for register-held vectors (constant
// register indices); over slot columns they are unrolled by 8, so a lane has
// eight independent loads in flight without keeping whole vectors live.
template <class Prob>
constexpr int kUnroll = Prob::kColumns ? 8 : Prob::N;

template <class Prob, class V>
RKMI_HD bool all_finite(const V& y) {
  constexpr int N = Prob::N, U = kUnroll<Prob>;
  bool ok = true;
#pragma unroll U
  for (int i = 0; i < N; ++i) ok = ok && crm::is_finite(y[i]);
  return ok;
}

template <class Prob, class VD, class VS>
RKMI_HD void copy(VD& d, const VS& s) {
  constexpr int N = Prob::N, U = kUnroll<Prob>;
#pragma unroll U
  for (int i = 0; i < N; ++i) d[i] = s[i];
}

// =========================================================================
// RKCK (Table 1 coefficients as nearest doubles of the printed fractions).
// =========================================================================
namespace ck {
constexpr double b21 = 1.0 / 5.0;
constexpr double b31 = 3.0 / 40.0, b32 = 9.0 / 40.0;
constexpr double b41 = 3.0 / 10.0, b42 = -9.0 / 10.0, b43 = 6.0 / 5.0;
constexpr double b51 = -11.0 / 54.0, b52 = 5.0 / 2.0, b53 = -70.0 / 27.0, b54 = 35.0 / 27.0;
constexpr double b61 = 1631.0 / 55296.0, b62 = 175.0 / 512.0, b63 = 575.0 / 13824.0,
                 b64 = 44275.0 / 110592.0, b65 = 253.0 / 4096.0;
constexpr double c1 = 37.0 / 378.0, c3 = 250.0 / 621.0, c4 = 125.0 / 594.0, c6 = 512.0 / 1771.0;
// c_i - c*_i, exact rational differences rounded once
constexpr double e1 = -277.0 / 64512.0, e3 = 6925.0 / 370944.0, e4 = -6925.0 / 202752.0,
                 e5 = -277.0 / 14336.0, e6 = 277.0 / 7084.0;
// the stage couplings and weights as tables (row i: stage i + 1), zero where
// Table 1 has no entry
constexpr double kB[6][5] = {{0.0, 0.0, 0.0, 0.0, 0.0},
                             {b21, 0.0, 0.0, 0.0, 0.0},
                             {b31, b32, 0.0, 0.0, 0.0},
                             {b41, b42, b43, 0.0, 0.0},
                             {b51, b52, b53, b54, 0.0},
                             {b61, b62, b63, b64, b65}};
constexpr double kC[6] = {c1, 0.0, c3, c4, 0.0, c6};
}  // namespace ck

// Observer of the stages of a step (the adjoint records them).  RKC: first()
// sees w_0 and mut_1, stage(j, ...) sees w_{j-1} with the coefficients of
// stage j before f(w_{j-1}) is formed; with kStopAtLast the step ends after
// stage(s, ...), without forming w_s.  RKCK: rkck_stage(i, z) sees the
// argument z_i of stage i = 2..6 before f(z_i) is formed.
struct NoSink {
  static constexpr bool kStopAtLast = false;
  template <class V>
  RKMI_HD void first(const V&, double) {}
  template <class V>
  RKMI_HD void stage(int, const V&, double, double, double, double) {}
  template <class V>
  RKMI_HD void rkck_stage(int, const V&) {}
};

// Observer of accepted steps (the adjoint's forward tape).
struct NoRec {
  template <class V>
  RKMI_HD void accept(double, int, const V&, int64_t) {}
};

// One trial step: k_1 = h F, k_i = h f(y + sum_j b_ij k_j); returns the
// fifth-order solution and the error estimate sum_i (c_i - c*_i) k_i.
template <class Prob, class Sink = NoSink>
RKMI_HD void rkck_trial(const typename Prob::Lane& L, const typename Prob::Params& prm,
                        const Vec<Prob>& y, const Vec<Prob>& F, double h, Vec<Prob>& yt,
                        Vec<Prob>& ye, double* slot, Sink* sink = nullptr) {
  constexpr int N = Prob::N, U = kUnroll<Prob>;
  Vec<Prob> k1 = work_vec<Prob>(slot, kCkK1), k2 = work_vec<Prob>(slot, kCkK2),
            k3 = work_vec<Prob>(slot, kCkK3), k4 = work_vec<Prob>(slot, kCkK4),
            k5 = work_vec<Prob>(slot, kCkK5), z = work_vec<Prob>(slot, kCkZ),
            f = work_vec<Prob>(slot, kCkFs);
#pragma unroll U
  for (int i = 0; i < N; ++i) {
    k1[i] = h * F[i];
    z[i] = y[i] + ck::b21 * k1[i];
  }
  if (sink) sink->rkck_stage(2, z);
  eval_rhs<Prob>(L, prm, z, f);
#pragma unroll U
  for (int i = 0; i < N; ++i) {
    k2[i] = h * f[i];
    z[i] = y[i] + ck::b31 * k1[i] + ck::b32 * k2[i];
  }
  if (sink) sink->rkck_stage(3, z);
  eval_rhs<Prob>(L, prm, z, f);
#pragma unroll U
  for (int i = 0; i < N; ++i) {
    k3[i] = h * f[i];
    z[i] = y[i] + ck::b41 * k1[i] + ck::b42 * k2[i] + ck::b43 * k3[i];
  }
  if (sink) sink->rkck_stage(4, z);
  eval_rhs<Prob>(L, prm, z, f);
#pragma unroll U
  for (int i = 0; i < N; ++i) {
    k4[i] = h * f[i];
    z[i] = y[i] + ck::b51 * k1[i] + ck::b52 * k2[i] + ck::b53 * k3[i] + ck::b54 * k4[i];
  }
  if (sink) sink->rkck_stage(5, z);
  eval_rhs<Prob>(L, prm, z, f);
#pragma unroll U
  for (int i = 0; i < N; ++i) {
    k5[i] = h * f[i];
    z[i] = y[i] + ck::b61 * k1[i] + ck::b62 * k2[i] + ck::b63 * k3[i] + ck::b64 * k4[i] +
           ck::b65 * k5[i];
  }
  if (sink) sink->rkck_stage(6, z);
  eval_rhs<Prob>(L, prm, z, f);
#pragma unroll U
  for (int i = 0; i < N; ++i) {
    const double k6 = h * f[i];
    yt[i] = y[i] + ck::c1 * k1[i] + ck::c3 * k3[i] + ck::c4 * k4[i] + ck::c6 * k6;
    ye[i] = 0.0 + ck::e1 * k1[i] + ck::e3 * k3[i] + ck::e4 * k4[i] + ck::e5 * k5[i] + ck::e6 * k6;
  }
}

// Integration state of one system under RKCK.
template <class Prob>
struct RkckState {
  Vec<Prob> y, F;
  double t, h;
  int64_t attempts;
  int32_t n_acc, n_rej, n_rhs, status;
  bool fvalid;
  double h_want;   // the step before the cut to the interval end
  bool cut;        // the last accepted step was cut
};

// Points the state's vectors at their slot columns (column storage only).
template <class Prob>
RKMI_HD void rkck_bind(RkckState<Prob>& S, double* slot) {
  if constexpr (Prob::kColumns) {
    S.y.p = col_ptr<Prob>(slot, kCkY);
    S.F.p = col_ptr<Prob>(slot, kCkF);
  } else {
    (void)S;
    (void)slot;
  }
}

template <class Prob>
RKMI_HD void rkck_begin(RkckState<Prob>& S, const Ctl& c) {
  S.t = c.t0;
  S.h = 0.5 * c.hmax;
  S.h_want = S.h;
  S.cut = false;
  S.fvalid = false;
  S.status = kSysOk;
  S.attempts = 0;
  S.n_acc = S.n_rej = S.n_rhs = 0;
}

// One attempted step of the RKCK driver (Sec. 3.1); returns true while the
// system still has to step (t < t1 and no failure).
template <class Prob, class Rec = NoRec>
RKMI_HD bool rkck_attempt(const typename Prob::Lane& L, const typename Prob::Params& prm,
                          const Ctl& c, RkckState<Prob>& S, double* slot, Rec* rec = nullptr) {
  constexpr int N = Prob::N, U = kUnroll<Prob>;
  if (S.attempts >= c.max_steps) {
    S.status = kSysMaxSteps;
    return false;
  }
  S.h_want = S.h;
  S.h = fmin(c.t1 - S.t, S.h);
  if (!S.fvalid) {
    eval_rhs<Prob>(L, prm, S.y, S.F);
    ++S.n_rhs;
    S.fvalid = true;
  }
  Vec<Prob> yt = work_vec<Prob>(slot, kCkYt), ye = work_vec<Prob>(slot, kCkYe);
  rkck_trial<Prob>(L, prm, S.y, S.F, S.h, yt, ye, slot);
  S.n_rhs += 5;
  ++S.attempts;
  // scaled error max_i |yerr_i / (|y_i| + |h F_i| + delta)| / rtol
  double err = 0.0;
  bool nan_flag = false;
#pragma unroll U
  for (int i = 0; i < N; ++i) {
    nan_flag = nan_flag || crm::is_nan(ye[i]);
    err = fmax(err, fabs(ye[i] / (fabs(S.y[i]) + fabs(S.h * S.F[i]) + c.delta)));
  }
  err = err / c.rtol;
  if ((err > 1.0) || crm::is_nan(err) || nan_flag) {
    ++S.n_rej;
    if (crm::is_nan(err) || nan_flag)
      S.h = S.h * kP1;
    else
      S.h = fmax(kSafety * S.h * crm::pow_minus_quarter(err), kP1 * S.h);
    if (!(S.h >= kRkckHmin)) {
      S.status = kSysHmin;
      return false;
    }
  } else {
    S.cut = S.h < S.h_want;
    S.t += S.h;
    const double hacc = S.h;
    const double hn = (err > kErrCon) ? kSafety * S.h * crm::pow_minus_fifth(err) : S.h * 5.0;
    S.h = fmax(kRkckHmin, fmin(c.hmax, hn));
    copy<Prob>(S.y, yt);
    ++S.n_acc;
    if (rec) rec->accept(hacc, 6, S.y, S.n_acc);
    S.fvalid = false;
    if (!all_finite<Prob>(S.y)) {
      S.status = kSysNonFinite;
      return false;
    }
  }
  return S.t < c.t1;
}

template <class Prob>
RKMI_HD void rkck_stats(const RkckState<Prob>& S, int32_t (&st)[kNStats]) {
  st[kStAccept] = S.n_acc;
  st[kStReject] = S.n_rej;
  st[kStRhs] = S.n_rhs;
  st[kStSrCalls] = 0;
  st[kStPowIters] = 0;
  st[kStMaxStages] = 6;
}

// =========================================================================
// RKC
// =========================================================================
constexpr double kKappa = 2.0 / 13.0;

// The coefficients of an s-stage step depend on s alone: omega_0 = 1 + kappa /
// s^2, omega_1 = T_s'(omega_0) / T_s''(omega_0) from the Chebyshev recurrence
// and its first two derivatives, b_j = T_j'' / T_j'^2 (b_0 = b_1 = b_2),
// a_j = 1 - b_j T_j, and per stage j >= 2 mu_j = 2 b_j omega_0 / b_{j-1},
// nu_j = -b_j / b_{j-2}, mut_j = 2 b_j omega_1 / b_{j-1}, gt_j = -a_{j-1} mut_j
// (the first stage uses mut_1 = b_1 omega_1).  RkcCoef runs the recurrences
// one stage at a time.
struct RkcStageCoef {
  double mu, nu, mut, gt, c0;   // c0 = 1 - mu - nu
};

struct RkcCoef {
  double w0 = 0.0, w1 = 0.0;
  double Tm2 = 1.0, Tm1 = 0.0, Dm2 = 0.0, Dm1 = 1.0, Em2 = 0.0, Em1 = 0.0;
  double bjm1 = 0.0, bjm2 = 0.0, ajm1 = 0.0;

  constexpr __host__ __device__ RkcCoef() {}     // unset (tabulated stage counts)
  constexpr __host__ __device__ explicit RkcCoef(int s) {
    w0 = 1.0 + kKappa / ((double)s * (double)s);
    double tm2 = 1.0, tm1 = w0, dm2 = 0.0, dm1 = 1.0, em2 = 0.0, em1 = 0.0;
    for (int j = 2; j <= s; ++j) {
      const double tj = 2.0 * w0 * tm1 - tm2;
      const double dj = 2.0 * tm1 + 2.0 * w0 * dm1 - dm2;
      const double ej = 4.0 * dm1 + 2.0 * w0 * em1 - em2;
      tm2 = tm1; tm1 = tj;
      dm2 = dm1; dm1 = dj;
      em2 = em1; em1 = ej;
    }
    w1 = dm1 / em1;
    Tm1 = w0;
    const double D2 = 2.0 * Tm1 + 2.0 * w0 * Dm1 - Dm2;
    const double E2 = 4.0 * Dm1 + 2.0 * w0 * Em1 - Em2;
    bjm1 = E2 / (D2 * D2);
    bjm2 = bjm1;
    ajm1 = 1.0 - bjm1 * w0;
  }
  constexpr __host__ __device__ double mut1() const { return bjm1 * w1; }
  // Coefficients of the next stage (j = 2, 3, ... in turn).
  constexpr __host__ __device__ RkcStageCoef next() {
    const double Tj = 2.0 * w0 * Tm1 - Tm2;
    const double Dj = 2.0 * Tm1 + 2.0 * w0 * Dm1 - Dm2;
    const double Ej = 4.0 * Dm1 + 2.0 * w0 * Em1 - Em2;
    const double bj = Ej / (Dj * Dj);
    RkcStageCoef c{};
    c.mu = 2.0 * bj * w0 / bjm1;
    c.nu = -bj / bjm2;
    c.mut = 2.0 * bj * w1 / bjm1;
    c.gt = -ajm1 * c.mut;
    c.c0 = 1.0 - c.mu - c.nu;
    ajm1 = 1.0 - bj * Tj;
    bjm2 = bjm1;
    bjm1 = bj;
    Tm2 = Tm1; Tm1 = Tj;
    Dm2 = Dm1; Dm1 = Dj;
    Em2 = Em1; Em1 = Ej;
    return c;
  }
};

// The coefficients for s <= kRkcTableS, evaluated by the compiler with the
// same IEEE operations in the same order (no contraction), hence the same
// bits as RkcCoef at run time; steps of up to kRkcTableS stages read them
// instead of forming ten divisions per step.
constexpr int kRkcTableS = 32;
constexpr int rkc_table_row(int s) { return (s - 2) * (s - 1) / 2; }   // stage 2 of s
struct RkcTable {
  double mut1[kRkcTableS + 1];
  RkcStageCoef st[rkc_table_row(kRkcTableS + 1)];
};
constexpr RkcTable make_rkc_table() {
  RkcTable t{};
  for (int s = 2; s <= kRkcTableS; ++s) {
    RkcCoef c(s);
    t.mut1[s] = c.mut1();
    for (int j = 2; j <= s; ++j) t.st[rkc_table_row(s) + j - 2] = c.next();
  }
  return t;
}
inline constexpr RkcTable kRkcTable = make_rkc_table();

// One RKC step of s stages from (y_n, F_n = f(y_n)) into y (Eqs. E:rkc0 - E:rkcs).
template <class Prob, class Sink = NoSink>
RKMI_HD void rkc_step(const typename Prob::Lane& L, const typename Prob::Params& prm,
                      const Vec<Prob>& yn, const Vec<Prob>& Fn, double h, int s, Vec<Prob>& y,
                      double* slot, Sink* sink = nullptr) {
  constexpr int N = Prob::N, U = kUnroll<Prob>;
  const bool tab = s <= kRkcTableS;
  RkcCoef cf;
  if (!tab) cf = RkcCoef(s);
  const int row = tab ? rkc_table_row(s) - 2 : 0;
  Vec<Prob> wjm2 = work_vec<Prob>(slot, kCWm2), f = work_vec<Prob>(slot, kCFs);
  const double mut1 = tab ? kRkcTable.mut1[s] : cf.mut1();
  const double mh1 = mut1 * h;           // mut_1 h
  if (sink) sink->first(yn, mut1);
#pragma unroll U
  for (int i = 0; i < N; ++i) {
    wjm2[i] = yn[i];
    y[i] = yn[i] + mh1 * Fn[i];          // y holds w_{j-1}
  }
  for (int j = 2; j <= s; ++j) {
    const RkcStageCoef k = tab ? kRkcTable.st[row + j] : cf.next();
    const double mh = k.mut * h, gh = k.gt * h;
    if (sink) {
      sink->stage(j, y, k.mu, k.nu, k.mut, k.gt);
      if (Sink::kStopAtLast && j == s) return;
    }
    eval_rhs<Prob>(L, prm, y, f);
#pragma unroll U
    for (int i = 0; i < N; ++i) {
      const double wj = k.c0 * yn[i] + k.mu * y[i] + k.nu * wjm2[i] + mh * f[i] + gh * Fn[i];
      wjm2[i] = y[i];
      y[i] = wj;
    }
  }
}

// Nonlinear power method (Appendix).  The eigenvector estimate v lives in
// slot column kCV between calls (and in registers during one when the system's
// vectors are register-held).  Returns 1.2 sigma and the iteration count.
template <class Prob>
RKMI_HD double spec_rad(const typename Prob::Lane& L, const typename Prob::Params& prm,
                        const Vec<Prob>& y, const Vec<Prob>& F, double hmax, int itmax,
                        double* slot, int& iters) {
  constexpr int N = Prob::N, U = kUnroll<Prob>;
  double* const vslot = col_ptr<Prob>(slot, kCV);
  Vec<Prob> v = work_vec<Prob>(slot, kCV), Fv = work_vec<Prob>(slot, kCFv);
  if constexpr (!Prob::kColumns) {
#pragma unroll U
    for (int i = 0; i < N; ++i) v[i] = vslot[i * kLdsStride];
  }
  const double sq = sqrt(kUround);
  const double small = 1.0 / hmax;
  double ynrm = 0.0, vnrm = 0.0;
#pragma unroll U
  for (int i = 0; i < N; ++i) {
    ynrm += y[i] * y[i];
    vnrm += v[i] * v[i];
  }
  ynrm = sqrt(ynrm);
  vnrm = sqrt(vnrm);
  double dynrm;
  if (ynrm != 0.0 && vnrm != 0.0) {
    dynrm = ynrm * sq;
    const double r = dynrm / vnrm;
#pragma unroll U
    for (int i = 0; i < N; ++i) v[i] = y[i] + v[i] * r;
  } else if (ynrm != 0.0) {
    dynrm = ynrm * sq;
#pragma unroll U
    for (int i = 0; i < N; ++i) v[i] = y[i] * (1.0 + sq);
  } else if (vnrm != 0.0) {
    dynrm = kUround;
    const double r = dynrm / vnrm;
#pragma unroll U
    for (int i = 0; i < N; ++i) v[i] = v[i] * r;
  } else {
    dynrm = kUround;
#pragma unroll U
    for (int i = 0; i < N; ++i) v[i] = kUround;
  }
  double sigma = 0.0;
  iters = itmax;
  for (int it = 1; it <= itmax; ++it) {
    eval_rhs<Prob>(L, prm, v, Fv);
    double d = 0.0;
#pragma unroll U
    for (int i = 0; i < N; ++i) d += (Fv[i] - F[i]) * (Fv[i] - F[i]);
    d = sqrt(d);
    const double sprev = sigma;
    sigma = d / dynrm;
    if (it >= 2 && fabs(sigma - sprev) <= fmax(sigma, small) * 0.01) {
#pragma unroll U
      for (int i = 0; i < N; ++i) v[i] = v[i] - y[i];
      iters = it;
      break;
    }
    if (d != 0.0) {
      const double r = dynrm / d;
#pragma unroll U
      for (int i = 0; i < N; ++i) v[i] = y[i] + (Fv[i] - F[i]) * r;
    } else {
      const int ind = it % N;
#pragma unroll U
      for (int i = 0; i < N; ++i)
        if (i == ind) v[i] = y[i] - (v[i] - y[i]);
    }
  }
  if constexpr (!Prob::kColumns) {
#pragma unroll U
    for (int i = 0; i < N; ++i) vslot[i * kLdsStride] = v[i];
  } else {
    (void)vslot;
  }
  return 1.2 * sigma;
}

// Stage count 1 + floor(sqrt(1 + 1.54 h sigma)), capped at mmax with the step
// shortened to (m^2 - 1) / (1.54 sigma).
RKMI_HD int rkc_stage_count(double& h, double sigma, int mmax) {
  const double x = sqrt(1.54 * h * sigma + 1.0);
  int m = (x < (double)mmax) ? 1 + (int)x : mmax + 1;
  if (m > mmax) {
    m = mmax;
    h = ((double)m * (double)m - 1.0) / (1.54 * sigma);
  }
  return m;
}

// Integration state of one system under RKC (the paper's work array: previous
// error and step, current step, spectral radius; the eigenvector is in the slot).
template <class Prob>
struct RkcState {
  Vec<Prob> yn, Fn;
  double t, h, h_prev, err_prev, sigma;
  double cbrt_err_prev;      // err_prev^(1/3), formed when err_prev was accepted
  int64_t nstep, attempts;
  int32_t sr_phase;          // nstep mod sr_period, kept step by step (no 64-bit modulo)
  int32_t n_acc, n_rej, n_rhs, n_sr, n_pow, max_m, status;
  bool first, have_prev;
  double h_want;   // the step before the cut to the interval end
  bool cut;        // the last accepted step was cut
};

template <class Prob>
RKMI_HD void rkc_bind(RkcState<Prob>& S, double* slot) {
  if constexpr (Prob::kColumns) {
    S.yn.p = col_ptr<Prob>(slot, kCYn);
    S.Fn.p = col_ptr<Prob>(slot, kCFn);
  } else {
    (void)S;
    (void)slot;
  }
}

// Restart state (Sec. 3): F_n = f(t0, y0), v = F_n, no step-size memory.
template <class Prob>
RKMI_HD void rkc_begin(const typename Prob::Lane& L, const typename Prob::Params& prm,
                       const Ctl& c, RkcState<Prob>& S, double* slot) {
  constexpr int N = Prob::N, U = kUnroll<Prob>;
  double* const vslot = col_ptr<Prob>(slot, kCV);
  S.t = c.t0;
  S.status = kSysOk;
  S.attempts = 0;
  S.n_acc = S.n_rej = S.n_rhs = S.n_sr = S.n_pow = S.max_m = 0;
  if (S.t < c.t1) {
    eval_rhs<Prob>(L, prm, S.yn, S.Fn);
    ++S.n_rhs;
  } else {
#pragma unroll U
    for (int i = 0; i < N; ++i) S.Fn[i] = 0.0;
  }
#pragma unroll U
  for (int i = 0; i < N; ++i) vslot[i * kLdsStride] = S.Fn[i];
  S.h = S.h_prev = S.err_prev = S.sigma = S.cbrt_err_prev = 0.0;
  S.h_want = 0.0;
  S.cut = false;
  S.nstep = 0;
  S.sr_phase = 0;
  S.first = true;
  S.have_prev = false;
}

// One attempted step of the RKC driver (Sec. 3.2); returns true while the
// system still has to step (t < t1 and no failure).
// A problem with an analytic Jacobian (Prob::kGershgorin, Prob::gershgorin(L,
// prm, y) = max_k sum_i |J_ki|, rows and sums in order).
template <class P, class = void>
struct HasGershgorin {
  static constexpr bool value = false;
};
template <class P>
struct HasGershgorin<P, std::void_t<decltype(P::kGershgorin)>> {
  static constexpr bool value = P::kGershgorin;
};

// The problem P with sigma from its Gershgorin bound: kernels of their own
// (the launchers pick them for sr_method kSrGershgorin), so the bound's
// registers do not weigh on the power-method kernels.
template <class P>
struct WithGershgorin : P {
  static constexpr bool kSigmaFromGershgorin = true;
};
template <class P, class = void>
struct SigmaFromGershgorin {
  static constexpr bool value = false;
};
template <class P>
struct SigmaFromGershgorin<P, std::void_t<decltype(P::kSigmaFromGershgorin)>> {
  static constexpr bool value = P::kSigmaFromGershgorin;
};

// sigma at y_n: the Gershgorin bound in the WithGershgorin kernels, else the
// nonlinear power method.
template <class Prob>
RKMI_HD void rkc_refresh_sigma(const typename Prob::Lane& L, const typename Prob::Params& prm,
                               const Ctl& c, RkcState<Prob>& S, double* slot) {
  if constexpr (SigmaFromGershgorin<Prob>::value) {
    S.sigma = Prob::gershgorin(L, prm, S.yn);
    ++S.n_sr;
    return;
  }
  int it;
  S.sigma = spec_rad<Prob>(L, prm, S.yn, S.Fn, c.hmax, c.sr_itmax, slot, it);
  ++S.n_sr;
  S.n_pow += it;
  S.n_rhs += it;
}

template <class Prob, class Rec = NoRec>
RKMI_HD bool rkc_attempt(const typename Prob::Lane& L, const typename Prob::Params& prm,
                         const Ctl& c, RkcState<Prob>& S, double* slot, Rec* rec = nullptr) {
  constexpr int N = Prob::N, U = kUnroll<Prob>;
  const double hmax = c.hmax, hmin = c.hmin_rkc;
  if (S.attempts >= c.max_steps) {
    S.status = kSysMaxSteps;
    return false;
  }
  S.h_want = S.h;
  if (1.1 * S.h >= fabs(c.t1 - S.t)) S.h = fabs(c.t1 - S.t);
  if (S.sr_phase == 0)            // nstep % sr_period == 0
    rkc_refresh_sigma<Prob>(L, prm, c, S, slot);
  Vec<Prob> y = work_vec<Prob>(slot, kCY), F1 = work_vec<Prob>(slot, kCF1);
  if (S.first) {
    // initial step from a trial Euler step of size min(hMax, 1/sigma)
    double h = hmax;
    if (S.sigma * h > 1.0) h = 1.0 / S.sigma;
    h = fmax(h, hmin);
#pragma unroll U
    for (int i = 0; i < N; ++i) y[i] = S.yn[i] + h * S.Fn[i];
    eval_rhs<Prob>(L, prm, y, F1);
    ++S.n_rhs;
    double e = 0.0;
#pragma unroll U
    for (int i = 0; i < N; ++i) {
      const double est = (F1[i] - S.Fn[i]) / (c.atol + c.rtol * fabs(S.yn[i]));
      e += est * est;
    }
    const double err0 = h * sqrt(e / (double)N);
    if (kP1 * h < hmax * sqrt(err0))
      h = fmax(kP1 * h / sqrt(err0), hmin);
    else
      h = hmax;
    S.h = h;
    S.first = false;
  }
  const int m = rkc_stage_count(S.h, S.sigma, c.mmax);
  S.max_m = max(S.max_m, m);
  rkc_step<Prob>(L, prm, S.yn, S.Fn, S.h, m, y, slot);
  eval_rhs<Prob>(L, prm, y, F1);
  S.n_rhs += m;
  ++S.attempts;
  double e = 0.0;
#pragma unroll U
  for (int i = 0; i < N; ++i) {
    double est = 0.8 * (S.yn[i] - y[i]) + 0.4 * S.h * (S.Fn[i] + F1[i]);
    est = est / (c.atol + c.rtol * fmax(fabs(y[i]), fabs(S.yn[i])));
    e += est * est;
  }
  const double err = sqrt(e / (double)N);
  if (err > 1.0 || !crm::is_finite(err)) {
    ++S.n_rej;
    S.h = crm::is_finite(err) ? 0.8 * S.h / crm::pow_third_one(err) : kP1 * S.h;
    rkc_refresh_sigma<Prob>(L, prm, c, S, slot);
    if (!(S.h >= hmin)) {
      S.status = kSysHmin;
      return false;
    }
  } else {
    S.cut = S.h < S.h_want;
    S.t += S.h;
    ++S.nstep;
    if (++S.sr_phase == c.sr_period) S.sr_phase = 0;
    ++S.n_acc;
    // err^(1/3) is kept for the next accepted step, where it is err_prev^(1/3);
    // err^(2/3) is the square of err^(1/3) (the double nearest 2/3 is twice
    // the one nearest 1/3)
    double cbrt_err, err23;
    crm::pow_third_pair(err, cbrt_err, err23);
    double fac = 10.0;
    if (!S.have_prev) {
      if (0.8 < fac * cbrt_err) fac = 0.8 / cbrt_err;
    } else {
      const double t1 = 0.8 * S.h * S.cbrt_err_prev;
      const double t2 = S.h_prev * err23;
      if (t1 < fac * t2) fac = t1 / t2;
    }
    S.err_prev = err;
    S.cbrt_err_prev = cbrt_err;
    S.h_prev = S.h;
    S.have_prev = true;
    copy<Prob>(S.yn, y);
    copy<Prob>(S.Fn, F1);
    if (rec) rec->accept(S.h, m, S.yn, S.nstep);
    S.h = S.h * fmax(kP1, fac);
    S.h = fmax(hmin, fmin(hmax, S.h));
    if (!all_finite<Prob>(S.yn)) {
      S.status = kSysNonFinite;
      return false;
    }
  }
  return S.t < c.t1;
}

template <class Prob>
RKMI_HD void rkc_stats(const RkcState<Prob>& S, int32_t (&st)[kNStats]) {
  st[kStAccept] = S.n_acc;
  st[kStReject] = S.n_rej;
  st[kStRhs] = S.n_rhs;
  st[kStSrCalls] = S.n_sr;
  st[kStPowIters] = S.n_pow;
  st[kStMaxStages] = S.max_m;
}

// A lane's integration of one system, in four parts: start (load state and
// parameters, per-system constants, restart state), attempt (one attempted
// step; false once the system is finished), finish (store; a null y1 stores
// only status and statistics).
template <class Prob, int Method, class Rec = NoRec>
struct Driver;

template <class Prob, class Rec>
struct Driver<Prob, kMethodRkck, Rec> {
  static constexpr int N = Prob::N, U = kUnroll<Prob>;
  typename Prob::Lane L;
  RkckState<Prob> S;
  Rec* rec = nullptr;
  RKMI_HD const Vec<Prob>& state() const { return S.y; }
  RKMI_HD int64_t accepted() const { return S.n_acc; }
  RKMI_HD bool start(const typename Prob::Params& prm, const Ctl& c, int64_t n, int64_t i,
                     const double* y0, const double* g, double* slot,
                     const double* carry = nullptr) {
    Prob::init(L, prm, g, i, n, slot);
    rkck_bind<Prob>(S, slot);
#pragma unroll U
    for (int k = 0; k < N; ++k) S.y[k] = y0[(int64_t)k * n + i];
    rkck_begin<Prob>(S, c);
    if (carry && carry[(int64_t)kCarryValid * n + i] != 0.0) {
      S.h = carry[(int64_t)kCarryH * n + i];
      S.h_want = S.h;
    }
    return S.t < c.t1;
  }
  RKMI_HD bool attempt(const typename Prob::Params& prm, const Ctl& c, double* slot) {
    return rkck_attempt<Prob, Rec>(L, prm, c, S, slot, rec);
  }
  RKMI_HD void finish(int64_t n, int64_t i, double* y1, int32_t* status, int32_t* stats,
                      double* carry = nullptr, const double* = nullptr) const {
    if (y1)
#pragma unroll U
      for (int k = 0; k < N; ++k) y1[(int64_t)k * n + i] = S.y[k];
    if (carry) {
      carry[(int64_t)kCarryValid * n + i] = S.status == kSysOk ? 1.0 : 0.0;
      carry[(int64_t)kCarryH * n + i] = S.cut ? S.h_want : S.h;
    }
    int32_t st[kNStats];
    rkck_stats(S, st);
    if (status) status[i] = S.status;
    if (stats)
#pragma unroll
      for (int r = 0; r < kNStats; ++r) stats[(int64_t)r * n + i] = st[r];
  }
};

template <class Prob, class Rec>
struct Driver<Prob, kMethodRkc, Rec> {
  static constexpr int N = Prob::N, U = kUnroll<Prob>;
  typename Prob::Lane L;
  RkcState<Prob> S;
  Rec* rec = nullptr;
  RKMI_HD const Vec<Prob>& state() const { return S.yn; }
  RKMI_HD int64_t accepted() const { return S.nstep; }
  RKMI_HD bool start(const typename Prob::Params& prm, const Ctl& c, int64_t n, int64_t i,
                     const double* y0, const double* g, double* slot,
                     const double* carry = nullptr) {
    Prob::init(L, prm, g, i, n, slot);
    rkc_bind<Prob>(S, slot);
#pragma unroll U
    for (int k = 0; k < N; ++k) S.yn[k] = y0[(int64_t)k * n + i];
    rkc_begin<Prob>(L, prm, c, S, slot);
    if (carry && carry[(int64_t)kCarryValid * n + i] != 0.0) {
      S.h = carry[(int64_t)kCarryH * n + i];
      S.h_prev = carry[(int64_t)kCarryHPrev * n + i];
      S.err_prev = carry[(int64_t)kCarryErrPrev * n + i];
      S.sigma = carry[(int64_t)kCarrySigma * n + i];
      S.nstep = (int64_t)carry[(int64_t)kCarryNstep * n + i];
      S.sr_phase = (int32_t)(S.nstep % c.sr_period);
      S.have_prev = carry[(int64_t)kCarryHavePrev * n + i] != 0.0;
      // err_prev^(1/3), as the controller formed it when err_prev was accepted
      S.cbrt_err_prev = S.have_prev ? crm::pow_third_one(S.err_prev) : 0.0;
      S.first = false;
      double* const vslot = col_ptr<Prob>(slot, kCV);
#pragma unroll U
      for (int k = 0; k < N; ++k) vslot[k * kLdsStride] = carry[(int64_t)(kCarryRows + k) * n + i];
    }
    return S.t < c.t1;
  }
  RKMI_HD bool attempt(const typename Prob::Params& prm, const Ctl& c, double* slot) {
    return rkc_attempt<Prob, Rec>(L, prm, c, S, slot, rec);
  }
  RKMI_HD void finish(int64_t n, int64_t i, double* y1, int32_t* status, int32_t* stats,
                      double* carry = nullptr, const double* slot = nullptr) const {
    if (y1)
#pragma unroll U
      for (int k = 0; k < N; ++k) y1[(int64_t)k * n + i] = S.yn[k];
    if (carry) {
      carry[(int64_t)kCarryValid * n + i] = S.status == kSysOk ? 1.0 : 0.0;
      carry[(int64_t)kCarryH * n + i] = S.cut ? S.h_want : S.h;
      carry[(int64_t)kCarryHPrev * n + i] = S.h_prev;
      carry[(int64_t)kCarryErrPrev * n + i] = S.err_prev;
      carry[(int64_t)kCarrySigma * n + i] = S.sigma;
      carry[(int64_t)kCarryNstep * n + i] = (double)S.nstep;
      carry[(int64_t)kCarryHavePrev * n + i] = S.have_prev ? 1.0 : 0.0;
      const double* const vslot = slot + (Prob::kLaneDoubles) * kLdsStride;
#pragma unroll U
      for (int k = 0; k < N; ++k) carry[(int64_t)(kCarryRows + k) * n + i] = vslot[k * kLdsStride];
    }
    int32_t st[kNStats];
    rkc_stats(S, st);
    if (status) status[i] = S.status;
    if (stats)
#pragma unroll
      for (int r = 0; r < kNStats; ++r) stats[(int64_t)r * n + i] = st[r];
  }
};

// One whole integration of system i by the lane.
template <class Prob, int Method>
RKMI_HD void integrate_system(const typename Prob::Params& prm, int64_t n, int64_t i,
                              const double* y0, double* y1, const double* g, const Ctl& c,
                              int32_t* status, int32_t* stats, double* slot,
                              double* carry = nullptr) {
  Driver<Prob, Method> D;
  if (D.start(prm, c, n, i, y0, g, slot, carry))
    while (D.attempt(prm, c, slot)) {
    }
  D.finish(n, i, y1, status, stats, carry, slot);
}

// =========================================================================
// Kernels
// =========================================================================

// The slot of this lane: in LDS for register-held systems, else in the
// workgroup's block of the column workspace (one block of slot_doubles
// columns per workgroup).
template <class Prob, int Method>
__device__ double* lane_slot(double* lds, double* cols) {
  if constexpr (Prob::kColumns)
    return cols + (int64_t)blockIdx.x * (slot_doubles<Prob, Method>() * kLdsStride) + threadIdx.x;
  else
    return lds + threadIdx.x;
}

template <class Prob, int Method>
constexpr int kernel_lds_doubles() {
  return (Prob::kColumns || slot_doubles<Prob, Method>() == 0) ? 1 : slot_doubles<Prob, Method>();
}

// Plain kernel: one lane per system, system i = global thread index (the
// paper's intDriver, Sec. 3), or order[global thread index] with an order map.
template <class Prob, int Method, bool kPilot = false>
__global__ __launch_bounds__(kLdsStride)
__attribute__((amdgpu_waves_per_eu(WavesPerEu<Prob>::value))) void plain_kernel(typename Prob::Params prm, int64_t n,
                                                           const double* y0,  // may alias y1
                                                           double* y1,
                                                           const double* __restrict__ g, Ctl c,
                                                           int32_t* __restrict__ status,
                                                           int32_t* __restrict__ stats,
                                                           double* cols,
                                                           const int32_t* __restrict__ order,
                                                           double* __restrict__ carry) {
  __shared__ double lds[kernel_lds_doubles<Prob, Method>() * kLdsStride];
  const int64_t q = (int64_t)blockIdx.x * kLdsStride + threadIdx.x;
  if (q >= n) return;
  const int64_t i = order ? (int64_t)order[q] : q;
  integrate_system<Prob, Method>(prm, n, i, y0, y1, g, c, status, stats,
                                 lane_slot<Prob, Method>(lds, cols), carry);
}

// Persistent loop of one wave over the systems of one queue: finished lanes
// take the next systems from a device-wide queue while the other lanes of
// their wave carry on, so lanes are not left idle behind the slowest system
// of a fixed group.  A wave refills once at least c.refill of its lanes are
// idle (or all its live lanes are): the systems started together form a
// cohort that runs its set-up and its periodic spectral-radius estimates in
// step, instead of each new lane running them alone.  The lanes taking work
// share one atomic add (wave-aggregated).  A lane retires once the queue is
// exhausted; the loop ends when all the wave's lanes have retired, so every
// wave leaves it.  Queue position q is system order[q] (q without a map).
// Called by all 64 lanes of the wave.
template <class Prob, int Method>
__device__ void persistent_loop(const typename Prob::Params& prm, int64_t n, const double* y0,
                                double* y1, const double* g, const Ctl& c, int32_t* status,
                                int32_t* stats, unsigned long long* queue, double* slot,
                                const int32_t* order, double* carry) {
  const int lane = threadIdx.x;
  Driver<Prob, Method> D;
  int64_t i = -1;
  bool active = false, retired = false;
  for (;;) {
    const bool idle = !active && !retired;
    const unsigned long long idle_mask = __ballot(idle);
    const bool refill =
        idle_mask && (__popcll(idle_mask) >= c.refill || !__ballot(active));
    const bool need = refill && idle;
    const unsigned long long need_mask = refill ? idle_mask : 0ull;
    if (need_mask) {
      const int leader = __ffsll((long long)need_mask) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(queue, (unsigned long long)__popcll(need_mask));
      base = __shfl(base, leader);
      if (need) {
        const unsigned long long below = need_mask & ((1ull << lane) - 1ull);
        const unsigned long long idx = base + (unsigned long long)__popcll(below);
        if (idx < (unsigned long long)n) {
          i = order ? (int64_t)order[idx] : (int64_t)idx;
          active = D.start(prm, c, n, i, y0, g, slot, carry);
          if (!active) D.finish(n, i, y1, status, stats, carry, slot);
        } else {
          retired = true;
        }
      }
    }
    if (!__ballot(!retired)) break;
    if (active && !D.attempt(prm, c, slot)) {
      D.finish(n, i, y1, status, stats, carry, slot);
      active = false;
    }
  }
}

// Persistent kernel: a grid sized to the machine running persistent_loop over
// the queue whose head, queue[0], must be zero at launch.  (kPilot only names
// the instance a cost-order pilot runs, here and in plain_kernel.)
template <class Prob, int Method, bool kPilot = false>
__global__ __launch_bounds__(kLdsStride)
__attribute__((amdgpu_waves_per_eu(WavesPerEu<Prob>::value))) void persistent_kernel(typename Prob::Params prm,
                                                                int64_t n, const double* y0,
                                                                double* y1,
                                                                const double* __restrict__ g,
                                                                Ctl c, int32_t* __restrict__ status,
                                                                int32_t* __restrict__ stats,
                                                                unsigned long long* queue,
                                                                double* cols,
                                                                const int32_t* __restrict__ order,
                                                                double* __restrict__ carry) {
  __shared__ double lds[kernel_lds_doubles<Prob, Method>() * kLdsStride];
  persistent_loop<Prob, Method>(prm, n, y0, y1, g, c, status, stats, queue,
                                lane_slot<Prob, Method>(lds, cols), order, carry);
}

}  // namespace rkmi
