// rk_device.hpp -- device-side RKCK / RKC drivers for one ODE system per lane.
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
//     max_steps attempts end the system with a status code.
//
// A problem type Prob supplies
//   static constexpr int N;              unknowns
//   struct Lane;                         per-system constants (registers)
//   using Params;                        uniform data passed by value
//   static void init(Lane&, const Params&, const double* g, int64_t i, int64_t n);
//   static void rhs(const Lane&, const Params&, const double (&y)[N], double (&f)[N]);
// Every right-hand side here is autonomous, so stage times are not formed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "crmath.hpp"
#include "rk_types.hpp"

namespace rkmi {

constexpr double kUround = 2.22e-16;
constexpr double kSafety = 0.9;
constexpr double kPGrow = -0.2;
constexpr double kPShrink = -0.25;
constexpr double kErrCon = 1.89e-4;
constexpr double kP1 = 0.1;
constexpr double kRkckHmin = 1.0e-20;

enum : int32_t { kSysOk = 0, kSysNonFinite = 1, kSysHmin = 2, kSysMaxSteps = 3 };
enum : int { kStAccept = 0, kStReject, kStRhs, kStSrCalls, kStPowIters, kStMaxStages, kNStats };

template <int N>
RKMI_HD bool all_finite(const double (&y)[N]) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < N; ++i) ok = ok && crm::is_finite(y[i]);
  return ok;
}

template <int N>
RKMI_HD void copy(double (&d)[N], const double (&s)[N]) {
#pragma unroll
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
}  // namespace ck

// One trial step: k_1 = h F, k_i = h f(y + sum_j b_ij k_j); returns the
// fifth-order solution and the error estimate sum_i (c_i - c*_i) k_i.
template <class Prob>
RKMI_HD void rkck_trial(const typename Prob::Lane& L,
                                           const typename Prob::Params& prm,
                                           const double (&y)[Prob::N], const double (&F)[Prob::N],
                                           double h, double (&yt)[Prob::N],
                                           double (&ye)[Prob::N]) {
  constexpr int N = Prob::N;
  double k1[N], k2[N], k3[N], k4[N], k5[N], z[N], f[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    k1[i] = h * F[i];
    z[i] = y[i] + ck::b21 * k1[i];
  }
  Prob::rhs(L, prm, z, f);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    k2[i] = h * f[i];
    z[i] = y[i] + ck::b31 * k1[i] + ck::b32 * k2[i];
  }
  Prob::rhs(L, prm, z, f);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    k3[i] = h * f[i];
    z[i] = y[i] + ck::b41 * k1[i] + ck::b42 * k2[i] + ck::b43 * k3[i];
  }
  Prob::rhs(L, prm, z, f);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    k4[i] = h * f[i];
    z[i] = y[i] + ck::b51 * k1[i] + ck::b52 * k2[i] + ck::b53 * k3[i] + ck::b54 * k4[i];
  }
  Prob::rhs(L, prm, z, f);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    k5[i] = h * f[i];
    z[i] = y[i] + ck::b61 * k1[i] + ck::b62 * k2[i] + ck::b63 * k3[i] + ck::b64 * k4[i] +
           ck::b65 * k5[i];
  }
  Prob::rhs(L, prm, z, f);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double k6 = h * f[i];
    yt[i] = y[i] + ck::c1 * k1[i] + ck::c3 * k3[i] + ck::c4 * k4[i] + ck::c6 * k6;
    ye[i] = 0.0 + ck::e1 * k1[i] + ck::e3 * k3[i] + ck::e4 * k4[i] + ck::e5 * k5[i] + ck::e6 * k6;
  }
}

// Per-lane RKCK integration of one system from t0 to t1 (in place on y).
template <class Prob>
__host__ __device__ int32_t rkck_integrate(const typename Prob::Lane& L, const typename Prob::Params& prm,
                                  const Ctl& c, double (&y)[Prob::N], int32_t (&st)[kNStats]) {
  constexpr int N = Prob::N;
  double F[N], yt[N], ye[N];
  double t = c.t0;
  double h = 0.5 * c.hmax;
  bool fvalid = false;
  int32_t status = kSysOk;
  int64_t attempts = 0;
  int32_t n_acc = 0, n_rej = 0, n_rhs = 0;
  while (t < c.t1) {
    if (attempts >= c.max_steps) {
      status = kSysMaxSteps;
      break;
    }
    h = fmin(c.t1 - t, h);
    if (!fvalid) {
      Prob::rhs(L, prm, y, F);
      ++n_rhs;
      fvalid = true;
    }
    rkck_trial<Prob>(L, prm, y, F, h, yt, ye);
    n_rhs += 5;
    ++attempts;
    // scaled error max_i |yerr_i / (|y_i| + |h F_i| + delta)| / rtol
    double err = 0.0;
    bool nan_flag = false;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      nan_flag = nan_flag || crm::is_nan(ye[i]);
      err = fmax(err, fabs(ye[i] / (fabs(y[i]) + fabs(h * F[i]) + c.delta)));
    }
    err = err / c.rtol;
    if ((err > 1.0) || crm::is_nan(err) || nan_flag) {
      ++n_rej;
      if (crm::is_nan(err) || nan_flag)
        h = h * kP1;
      else
        h = fmax(kSafety * h * crm::cr_pow(err, kPShrink), kP1 * h);
      if (!(h >= kRkckHmin)) {
        status = kSysHmin;
        break;
      }
    } else {
      t += h;
      double hn = (err > kErrCon) ? kSafety * h * crm::cr_pow(err, kPGrow) : h * 5.0;
      h = fmax(kRkckHmin, fmin(c.hmax, hn));
      copy(y, yt);
      ++n_acc;
      fvalid = false;
      if (!all_finite(y)) {
        status = kSysNonFinite;
        break;
      }
    }
  }
  st[kStAccept] = n_acc;
  st[kStReject] = n_rej;
  st[kStRhs] = n_rhs;
  st[kStSrCalls] = 0;
  st[kStPowIters] = 0;
  st[kStMaxStages] = 6;
  return status;
}

// =========================================================================
// RKC
// =========================================================================
constexpr double kKappa = 2.0 / 13.0;

// omega_0 = 1 + kappa / s^2 and omega_1 = T_s'(omega_0) / T_s''(omega_0) from
// the Chebyshev recurrence and its first two derivatives.
RKMI_HD void rkc_omegas(int s, double& w0, double& w1) {
  w0 = 1.0 + kKappa / ((double)s * (double)s);
  double Tm2 = 1.0, Tm1 = w0, Dm2 = 0.0, Dm1 = 1.0, Em2 = 0.0, Em1 = 0.0;
  for (int j = 2; j <= s; ++j) {
    double Tj = 2.0 * w0 * Tm1 - Tm2;
    double Dj = 2.0 * Tm1 + 2.0 * w0 * Dm1 - Dm2;
    double Ej = 4.0 * Dm1 + 2.0 * w0 * Em1 - Em2;
    Tm2 = Tm1; Tm1 = Tj;
    Dm2 = Dm1; Dm1 = Dj;
    Em2 = Em1; Em1 = Ej;
  }
  w1 = Dm1 / Em1;
}

// One RKC step of s stages from (y_n, F_n = f(y_n)) into y (Eqs. E:rkc0 - E:rkcs);
// the coefficients b_j, mu_j, nu_j, mut_j, gt_j are formed stage by stage.
template <class Prob>
RKMI_HD void rkc_step(const typename Prob::Lane& L,
                                         const typename Prob::Params& prm,
                                         const double (&yn)[Prob::N], const double (&Fn)[Prob::N],
                                         double h, int s, double (&y)[Prob::N]) {
  constexpr int N = Prob::N;
  double w0, w1;
  rkc_omegas(s, w0, w1);
  // j = 2 values of the recurrence: T_2 = 2 w0^2 - 1, T_2' = 4 w0, T_2'' = 4
  double Tm2 = 1.0, Tm1 = w0, Dm2 = 0.0, Dm1 = 1.0, Em2 = 0.0, Em1 = 0.0;
  double b2;
  {
    double T2 = 2.0 * w0 * Tm1 - Tm2;
    double D2 = 2.0 * Tm1 + 2.0 * w0 * Dm1 - Dm2;
    double E2 = 4.0 * Dm1 + 2.0 * w0 * Em1 - Em2;
    (void)T2;
    b2 = E2 / (D2 * D2);
  }
  double bjm1 = b2, bjm2 = b2;           // b_1 = b_0 = b_2
  double ajm1 = 1.0 - bjm1 * w0;         // a_1 = 1 - b_1 T_1
  double wjm1[N], wjm2[N], f[N];
  const double mh1 = (bjm1 * w1) * h;    // mut_1 h
#pragma unroll
  for (int i = 0; i < N; ++i) {
    wjm2[i] = yn[i];
    wjm1[i] = yn[i] + mh1 * Fn[i];
  }
  for (int j = 2; j <= s; ++j) {
    double Tj = 2.0 * w0 * Tm1 - Tm2;
    double Dj = 2.0 * Tm1 + 2.0 * w0 * Dm1 - Dm2;
    double Ej = 4.0 * Dm1 + 2.0 * w0 * Em1 - Em2;
    double bj = Ej / (Dj * Dj);
    double mu = 2.0 * bj * w0 / bjm1;
    double nu = -bj / bjm2;
    double mut = 2.0 * bj * w1 / bjm1;
    double gt = -ajm1 * mut;
    double c0 = 1.0 - mu - nu;
    double mh = mut * h, gh = gt * h;
    Prob::rhs(L, prm, wjm1, f);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double wj = c0 * yn[i] + mu * wjm1[i] + nu * wjm2[i] + mh * f[i] + gh * Fn[i];
      wjm2[i] = wjm1[i];
      wjm1[i] = wj;
    }
    ajm1 = 1.0 - bj * Tj;
    bjm2 = bjm1;
    bjm1 = bj;
    Tm2 = Tm1; Tm1 = Tj;
    Dm2 = Dm1; Dm1 = Dj;
    Em2 = Em1; Em1 = Ej;
  }
  copy(y, wjm1);
}

// Nonlinear power method (Appendix): v holds the eigenvector estimate between
// calls; Fv is scratch.  Returns 1.2 sigma and the iteration count.
template <class Prob>
RKMI_HD double spec_rad(const typename Prob::Lane& L,
                                           const typename Prob::Params& prm,
                                           const double (&y)[Prob::N], const double (&F)[Prob::N],
                                           double hmax, int itmax, double (&v)[Prob::N],
                                           int& iters) {
  constexpr int N = Prob::N;
  double Fv[N];
  const double sq = sqrt(kUround);
  const double small = 1.0 / hmax;
  double ynrm = 0.0, vnrm = 0.0;
#pragma unroll
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
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = y[i] + v[i] * r;
  } else if (ynrm != 0.0) {
    dynrm = ynrm * sq;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = y[i] * (1.0 + sq);
  } else if (vnrm != 0.0) {
    dynrm = kUround;
    const double r = dynrm / vnrm;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = v[i] * r;
  } else {
    dynrm = kUround;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = kUround;
  }
  double sigma = 0.0;
  iters = itmax;
  for (int it = 1; it <= itmax; ++it) {
    Prob::rhs(L, prm, v, Fv);
    double d = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) d += (Fv[i] - F[i]) * (Fv[i] - F[i]);
    d = sqrt(d);
    const double sprev = sigma;
    sigma = d / dynrm;
    if (it >= 2 && fabs(sigma - sprev) <= fmax(sigma, small) * 0.01) {
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = v[i] - y[i];
      iters = it;
      break;
    }
    if (d != 0.0) {
      const double r = dynrm / d;
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = y[i] + (Fv[i] - F[i]) * r;
    } else {
      const int ind = it % N;
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (i == ind) v[i] = y[i] - (v[i] - y[i]);
    }
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

// Per-lane RKC integration of one system from t0 to t1 (in place on y).
template <class Prob>
__host__ __device__ int32_t rkc_integrate(const typename Prob::Lane& L, const typename Prob::Params& prm,
                                 const Ctl& c, double (&y)[Prob::N], int32_t (&st)[kNStats]) {
  constexpr int N = Prob::N;
  double yn[N], Fn[N], F1[N], v[N];
  double t = c.t0;
  const double hmax = c.hmax, hmin = c.hmin_rkc;
  int32_t status = kSysOk;
  int64_t attempts = 0;
  int32_t n_acc = 0, n_rej = 0, n_rhs = 0, n_sr = 0, n_pow = 0, max_m = 0;
  copy(yn, y);
  if (t < c.t1) {
    Prob::rhs(L, prm, yn, Fn);
    ++n_rhs;
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) Fn[i] = 0.0;
  }
  copy(v, Fn);
  double h = 0.0, h_prev = 0.0, err_prev = 0.0, sigma = 0.0;
  int64_t nstep = 0;
  bool first = true, have_prev = false;
  while (t < c.t1) {
    if (attempts >= c.max_steps) {
      status = kSysMaxSteps;
      break;
    }
    if (1.1 * h >= fabs(c.t1 - t)) h = fabs(c.t1 - t);
    if (nstep % c.sr_period == 0) {
      int it;
      sigma = spec_rad<Prob>(L, prm, yn, Fn, hmax, c.sr_itmax, v, it);
      ++n_sr;
      n_pow += it;
      n_rhs += it;
    }
    if (first) {
      // initial step from a trial Euler step of size min(hMax, 1/sigma)
      h = hmax;
      if (sigma * h > 1.0) h = 1.0 / sigma;
      h = fmax(h, hmin);
#pragma unroll
      for (int i = 0; i < N; ++i) y[i] = yn[i] + h * Fn[i];
      Prob::rhs(L, prm, y, F1);
      ++n_rhs;
      double e = 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const double est = (F1[i] - Fn[i]) / (c.atol + c.rtol * fabs(yn[i]));
        e += est * est;
      }
      const double err0 = h * sqrt(e / (double)N);
      if (kP1 * h < hmax * sqrt(err0))
        h = fmax(kP1 * h / sqrt(err0), hmin);
      else
        h = hmax;
      first = false;
    }
    const int m = rkc_stage_count(h, sigma, c.mmax);
    max_m = max(max_m, m);
    rkc_step<Prob>(L, prm, yn, Fn, h, m, y);
    Prob::rhs(L, prm, y, F1);
    n_rhs += m;
    ++attempts;
    double e = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double est = 0.8 * (yn[i] - y[i]) + 0.4 * h * (Fn[i] + F1[i]);
      est = est / (c.atol + c.rtol * fmax(fabs(y[i]), fabs(yn[i])));
      e += est * est;
    }
    const double err = sqrt(e / (double)N);
    if (err > 1.0 || !crm::is_finite(err)) {
      ++n_rej;
      h = crm::is_finite(err) ? 0.8 * h / crm::cr_pow(err, 1.0 / 3.0) : kP1 * h;
      int it;
      sigma = spec_rad<Prob>(L, prm, yn, Fn, hmax, c.sr_itmax, v, it);
      ++n_sr;
      n_pow += it;
      n_rhs += it;
      if (!(h >= hmin)) {
        status = kSysHmin;
        break;
      }
    } else {
      t += h;
      ++nstep;
      ++n_acc;
      double fac = 10.0;
      if (!have_prev) {
        const double t2 = crm::cr_pow(err, 1.0 / 3.0);
        if (0.8 < fac * t2) fac = 0.8 / t2;
      } else {
        const double t1 = 0.8 * h * crm::cr_pow(err_prev, 1.0 / 3.0);
        const double t2 = h_prev * crm::cr_pow(err, 2.0 / 3.0);
        if (t1 < fac * t2) fac = t1 / t2;
      }
      err_prev = err;
      h_prev = h;
      have_prev = true;
      copy(yn, y);
      copy(Fn, F1);
      h = h * fmax(kP1, fac);
      h = fmax(hmin, fmin(hmax, h));
      if (!all_finite(yn)) {
        status = kSysNonFinite;
        break;
      }
    }
  }
  copy(y, yn);
  st[kStAccept] = n_acc;
  st[kStReject] = n_rej;
  st[kStRhs] = n_rhs;
  st[kStSrCalls] = n_sr;
  st[kStPowIters] = n_pow;
  st[kStMaxStages] = max_m;
  return status;
}

// =========================================================================
// Plain kernels: one lane per system, struct-of-arrays loads and stores.
// =========================================================================
template <class Prob, int Method>
__global__ __launch_bounds__(64) void plain_kernel(typename Prob::Params prm, int64_t n,
                                                   const double* y0,  // may alias y1
                                                   double* y1,
                                                   const double* __restrict__ g, Ctl c,
                                                   int32_t* __restrict__ status,
                                                   int32_t* __restrict__ stats) {
  constexpr int N = Prob::N;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  typename Prob::Lane L;
  Prob::init(L, prm, g, i, n);
  double y[N];
#pragma unroll
  for (int k = 0; k < N; ++k) y[k] = y0[(int64_t)k * n + i];
  int32_t st[kNStats];
  int32_t s = (Method == 0) ? rkck_integrate<Prob>(L, prm, c, y, st)
                            : rkc_integrate<Prob>(L, prm, c, y, st);
#pragma unroll
  for (int k = 0; k < N; ++k) y1[(int64_t)k * n + i] = y[k];
  if (status) status[i] = s;
  if (stats) {
#pragma unroll
    for (int r = 0; r < kNStats; ++r) stats[(int64_t)r * n + i] = st[r];
  }
}

}  // namespace rkmi
