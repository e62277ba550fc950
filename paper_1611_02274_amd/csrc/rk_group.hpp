// rk_group.hpp -- RKCK / RKC with L lanes of a wave sharing one system.
//
// For networks whose vectors do not fit one lane's registers, a group of L
// consecutive lanes integrates one system: lane r of the group owns the
// unknowns k = m L + r (m < S) of every vector and the reactions
// j = m L + r (m < R) with their rate constants, all in registers.  The
// right-hand side exchanges concentrations and rates of progress through the
// group's LDS area:
//   1. owners write C_k = (rho Y_k) / W_k; lane 0 forms [M] = sum_k C_k;
//   2. owners of reaction j write q_j = k_f prod_R C - k_r prod_P C and -q_j;
//   3. owners of species k sum their signed q_j in reaction order, then
//      f_k = (W_k omega_k) / rho,
// which is the per-system evaluation order, so results equal the one-lane
// kernels and the oracle bit for bit.  Weighted norms are formed in species
// order from the group's LDS scratch by every lane, so the step-size
// controller runs identically (and redundantly) in the L lanes.  The groups
// of a wave hold different systems and may diverge like lanes do.
//
// A group problem GP supplies N, NR, kL (lanes per system), S, R, the LDS
// layout (kOffC, kOffQ, kOffRed, kLdsPerSystem), the tables kRx (packed
// species indices of each reaction, [M] as index N), kTermOff / kTerms
// (signed rate indices of each species' sum in reaction order), Params,
// Lane, init(Lane&, prm, g, i, n, x); species of slot m of
// lane r: kSp[m L + r] (-1 for none), chosen so each slot's term lists have
// similar lengths; each lane's term codes are packed in its registers.
#pragma once

#include "rk_device.hpp"

namespace rkmi {

// The variant of a problem the persistent ragged kernel runs: the problem
// itself, or its group variant where one is generated.
template <class Prob>
struct FastVariant {
  using type = Prob;
};

// A lane's place in its group and the species it owns (slot m holds species
// sp[m], or none when sp[m] < 0).
template <class GP>
struct Grp {
  int r;                     // position in the group
  double* lds;               // the group's LDS area
  unsigned long long mask;   // the group's lanes in the wave
  int sp[GP::S];
};

// Orders the group's LDS accesses (one wave per workgroup: no barrier wait).
__device__ inline void group_sync() { __syncthreads(); }

// Hides a value from the optimizer at this point, so the LDS addresses formed
// from a lane's constant tables are recomputed in each evaluation instead of
// being hoisted out of the integration loop into ~100 extra live registers.
__device__ inline void opaque(uint32_t& v) { asm volatile("" : "+v"(v)); }

template <class GP>
__device__ inline bool owns(const Grp<GP>& x, int m) {
  return x.sp[m] >= 0;
}

// sum_k t_k over k = 0..N-1 in order, t_k held by the owners (slot m of lane
// r holds k = m L + r); every lane of the group gets the same value.
template <class GP>
__device__ double group_sum(const Grp<GP>& x, const double (&t)[GP::S]) {
  double* red = x.lds + GP::kOffRed;
#pragma unroll
  for (int m = 0; m < GP::S; ++m)
    if (owns<GP>(x, m)) red[x.sp[m]] = t[m];
  group_sync();
  double s = 0.0;
#pragma unroll 8
  for (int k = 0; k < GP::N; ++k) s += red[k];
  group_sync();
  return s;
}

// max(0, max_k t_k) with fmax, t_k >= +0 or NaN: the largest non-NaN value (or
// 0), which no order of the fmax operations changes.  Each lane folds its owned
// slots from 0 (so no partial result is NaN), then the group's lanes combine
// in a butterfly of register exchanges (the group is kL aligned lanes, kL a
// power of two, and reaches this point together).
template <class GP>
__device__ double group_fmax(const Grp<GP>& x, const double (&t)[GP::S]) {
  static_assert((GP::kL & (GP::kL - 1)) == 0 && GP::kL <= 64, "group width");
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < GP::S; ++m)
    if (owns<GP>(x, m)) s = fmax(s, t[m]);
#pragma unroll
  for (int o = 1; o < GP::kL; o <<= 1) s = fmax(s, __shfl_xor(s, o, GP::kL));
  return s;
}

// True on every lane of the group when `flag` holds on one of its lanes.
template <class GP>
__device__ inline bool group_any(const Grp<GP>& x, bool flag) {
  return (__ballot(flag) & x.mask) != 0;
}

template <class GP>
__device__ bool group_all_finite(const Grp<GP>& x, const double (&y)[GP::S]) {
  bool bad = false;
#pragma unroll
  for (int m = 0; m < GP::S; ++m) bad = bad || (owns<GP>(x, m) && !crm::is_finite(y[m]));
  return !group_any(x, bad);
}

// A group problem with a right-hand side of its own (GP::kOwnRhs, GP::rhs)
// rather than the mass-action exchange below.
template <class GP, class = void>
struct GroupOwnRhs {
  static constexpr bool value = false;
};
template <class GP>
struct GroupOwnRhs<GP, std::void_t<decltype(GP::kOwnRhs)>> {
  static constexpr bool value = GP::kOwnRhs;
};

template <class GP>
__device__ void group_rhs_mass_action(const typename GP::Lane& L, const Grp<GP>& x,
                                      const double (&y)[GP::S], double (&f)[GP::S]);

// Right-hand side of the group's system at y (owned slots) into f.
template <class GP>
__device__ void group_rhs(const typename GP::Lane& L, const Grp<GP>& x, const double (&y)[GP::S],
                          double (&f)[GP::S]) {
  if constexpr (GroupOwnRhs<GP>::value)
    GP::rhs(L, x, y, f);
  else
    group_rhs_mass_action<GP>(L, x, y, f);
}

// Mass action: concentrations, [M] and rates of progress exchanged through
// the group's LDS area (the scheme in the header comment).
template <class GP>
__device__ void group_rhs_mass_action(const typename GP::Lane& L, const Grp<GP>& x,
                                      const double (&y)[GP::S], double (&f)[GP::S]) {
  constexpr int N = GP::N, NR = GP::NR, LL = GP::kL;
  (void)LL;
  double* const C = x.lds + GP::kOffC;
  double* const Q = x.lds + GP::kOffQ;
#pragma unroll
  for (int m = 0; m < GP::S; ++m)
    if (owns<GP>(x, m)) C[x.sp[m]] = (L.rho * y[m]) * L.iW[m];
  group_sync();
  if (x.r == 0) {
    double M = 0.0;
#pragma unroll 8
    for (int k = 0; k < N; ++k) M += C[k];
    C[N] = M;
  }
  group_sync();
#pragma unroll
  for (int m = 0; m < GP::R; ++m) {
    const int j = m * LL + x.r;
    if (j < NR) {
      uint32_t code = L.rx[m];
      opaque(code);
      const double ca = C[code & 0xffu], cb = C[(code >> 8) & 0xffu];
      const double cc = C[(code >> 16) & 0xffu], cd = C[code >> 24];
      const double q = (L.kf[m] * ca) * cb - (L.kr[m] * cc) * cd;
      Q[j] = q;
      Q[NR + 1 + j] = -q;
    }
    // bound how far the scheduler moves loads ahead (register pressure)
    if (m % 2 == 1) __builtin_amdgcn_sched_barrier(0);
  }
  group_sync();
#pragma unroll
  for (int m = 0; m < GP::S; ++m) {
    double om = 0.0;
#pragma unroll
    for (int t = GP::kTermOff[m]; t < GP::kTermOff[m + 1]; ++t) {
      // term t: kTermBits-bit index into the signed rates, packed
      // kTermsPerWord to a register; om - q is formed as om + (-q)
      uint32_t word = L.tc[t / GP::kTermsPerWord];
      if (t % GP::kTermsPerWord == 0) opaque(word);
      const uint32_t code = (word >>
                             ((t % GP::kTermsPerWord) * GP::kTermBits)) &
                            ((1u << GP::kTermBits) - 1u);
      om = om + Q[code];
      if (t % 4 == 3) __builtin_amdgcn_sched_barrier(0);
    }
    f[m] = owns<GP>(x, m) ? (L.W[m] * om) * L.irho : 0.0;
  }
}

template <class GP>
__device__ void gcopy(double (&d)[GP::S], const double (&s)[GP::S]) {
#pragma unroll
  for (int m = 0; m < GP::S; ++m) d[m] = s[m];
}

// ------------------------------------------------------------------- RKCK
template <class GP>
struct GRkck {
  static constexpr int S = GP::S;
  typename GP::Lane L;
  double y[S], F[S];
  double t, h, h_want;
  int64_t attempts;
  int32_t n_acc, n_rej, n_rhs, status;
  bool fvalid, cut;

  __device__ void begin(const Ctl& c) {
    t = c.t0;
    h = 0.5 * c.hmax;
    h_want = h;
    cut = false;
    fvalid = false;
    status = kSysOk;
    attempts = 0;
    n_acc = n_rej = n_rhs = 0;
  }

  __device__ bool attempt(const Grp<GP>& x, const Ctl& c) {
    if (attempts >= c.max_steps) {
      status = kSysMaxSteps;
      return false;
    }
    h_want = h;
    h = fmin(c.t1 - t, h);
    if (!fvalid) {
      group_rhs<GP>(L, x, y, F);
      ++n_rhs;
      fvalid = true;
    }
    double k1[S], k2[S], k3[S], k4[S], k5[S], z[S], f[S], yt[S], ye[S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
      k1[i] = h * F[i];
      z[i] = y[i] + ck::b21 * k1[i];
    }
    group_rhs<GP>(L, x, z, f);
#pragma unroll
    for (int i = 0; i < S; ++i) {
      k2[i] = h * f[i];
      z[i] = y[i] + ck::b31 * k1[i] + ck::b32 * k2[i];
    }
    group_rhs<GP>(L, x, z, f);
#pragma unroll
    for (int i = 0; i < S; ++i) {
      k3[i] = h * f[i];
      z[i] = y[i] + ck::b41 * k1[i] + ck::b42 * k2[i] + ck::b43 * k3[i];
    }
    group_rhs<GP>(L, x, z, f);
#pragma unroll
    for (int i = 0; i < S; ++i) {
      k4[i] = h * f[i];
      z[i] = y[i] + ck::b51 * k1[i] + ck::b52 * k2[i] + ck::b53 * k3[i] + ck::b54 * k4[i];
    }
    group_rhs<GP>(L, x, z, f);
#pragma unroll
    for (int i = 0; i < S; ++i) {
      k5[i] = h * f[i];
      z[i] = y[i] + ck::b61 * k1[i] + ck::b62 * k2[i] + ck::b63 * k3[i] + ck::b64 * k4[i] +
             ck::b65 * k5[i];
    }
    group_rhs<GP>(L, x, z, f);
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const double k6 = h * f[i];
      yt[i] = y[i] + ck::c1 * k1[i] + ck::c3 * k3[i] + ck::c4 * k4[i] + ck::c6 * k6;
      ye[i] = 0.0 + ck::e1 * k1[i] + ck::e3 * k3[i] + ck::e4 * k4[i] + ck::e5 * k5[i] +
              ck::e6 * k6;
    }
    n_rhs += 5;
    ++attempts;
    double a[S];
    bool nan_flag = false;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      nan_flag = nan_flag || (owns<GP>(x, i) && crm::is_nan(ye[i]));
      a[i] = fabs(ye[i] / (fabs(y[i]) + fabs(h * F[i]) + c.delta));
    }
    nan_flag = group_any(x, nan_flag);
    double err = group_fmax<GP>(x, a);
    err = err / c.rtol;
    if ((err > 1.0) || crm::is_nan(err) || nan_flag) {
      ++n_rej;
      if (crm::is_nan(err) || nan_flag)
        h = h * kP1;
      else
        h = fmax(kSafety * h * crm::pow_minus_quarter(err), kP1 * h);
      if (!(h >= kRkckHmin)) {
        status = kSysHmin;
        return false;
      }
    } else {
      cut = h < h_want;
      t += h;
      const double hn = (err > kErrCon) ? kSafety * h * crm::pow_minus_fifth(err) : h * 5.0;
      h = fmax(kRkckHmin, fmin(c.hmax, hn));
      gcopy<GP>(y, yt);
      ++n_acc;
      fvalid = false;
      if (!group_all_finite<GP>(x, y)) {
        status = kSysNonFinite;
        return false;
      }
    }
    return t < c.t1;
  }

  __device__ void stats(int32_t (&st)[kNStats]) const {
    st[kStAccept] = n_acc;
    st[kStReject] = n_rej;
    st[kStRhs] = n_rhs;
    st[kStSrCalls] = 0;
    st[kStPowIters] = 0;
    st[kStMaxStages] = 6;
  }
  __device__ const double (&state() const)[S] { return y; }
  __device__ double (&state())[S] { return y; }
  // carried controller state (rows of the carry array), as the one-lane driver
  __device__ void load_carry(const Grp<GP>&, const Ctl&, const double* carry, int64_t n,
                             int64_t i) {
    h = carry[(int64_t)kCarryH * n + i];
    h_want = h;
  }
  __device__ void store_carry(const Grp<GP>& x, double* carry, int64_t n, int64_t i) const {
    if (x.r != 0) return;
    carry[(int64_t)kCarryValid * n + i] = status == kSysOk ? 1.0 : 0.0;
    carry[(int64_t)kCarryH * n + i] = cut ? h_want : h;
  }
};

// -------------------------------------------------------------------- RKC
template <class GP>
struct GRkc {
  static constexpr int S = GP::S, N = GP::N;
  typename GP::Lane L;
  double yn[S], Fn[S], v[S];
  double t, h, h_prev, err_prev, sigma, cbrt_err_prev, h_want;
  int64_t nstep, attempts;
  int32_t sr_phase;          // nstep mod sr_period
  int32_t n_acc, n_rej, n_rhs, n_sr, n_pow, max_m, status;
  bool first, have_prev, cut;

  __device__ void begin(const Grp<GP>& x, const Ctl& c) {
    t = c.t0;
    status = kSysOk;
    attempts = 0;
    n_acc = n_rej = n_rhs = n_sr = n_pow = max_m = 0;
    if (t < c.t1) {
      group_rhs<GP>(L, x, yn, Fn);
      ++n_rhs;
    } else {
#pragma unroll
      for (int i = 0; i < S; ++i) Fn[i] = 0.0;
    }
    gcopy<GP>(v, Fn);
    h = h_prev = err_prev = sigma = cbrt_err_prev = h_want = 0.0;
    nstep = 0;
    sr_phase = 0;
    first = true;
    have_prev = false;
    cut = false;
  }

  // Nonlinear power method (Appendix), as spec_rad.
  __device__ double spec_rad(const Grp<GP>& x, double hmax, int itmax, int& iters) {
    double Fv[S], t2[S];
    const double sq = sqrt(kUround);
    const double small = 1.0 / hmax;
#pragma unroll
    for (int i = 0; i < S; ++i) t2[i] = yn[i] * yn[i];
    double ynrm = group_sum<GP>(x, t2);
#pragma unroll
    for (int i = 0; i < S; ++i) t2[i] = v[i] * v[i];
    double vnrm = group_sum<GP>(x, t2);
    ynrm = sqrt(ynrm);
    vnrm = sqrt(vnrm);
    double dynrm;
    if (ynrm != 0.0 && vnrm != 0.0) {
      dynrm = ynrm * sq;
      const double r = dynrm / vnrm;
#pragma unroll
      for (int i = 0; i < S; ++i) v[i] = yn[i] + v[i] * r;
    } else if (ynrm != 0.0) {
      dynrm = ynrm * sq;
#pragma unroll
      for (int i = 0; i < S; ++i) v[i] = yn[i] * (1.0 + sq);
    } else if (vnrm != 0.0) {
      dynrm = kUround;
      const double r = dynrm / vnrm;
#pragma unroll
      for (int i = 0; i < S; ++i) v[i] = v[i] * r;
    } else {
      dynrm = kUround;
#pragma unroll
      for (int i = 0; i < S; ++i) v[i] = owns<GP>(x, i) ? kUround : 0.0;
    }
    double sig = 0.0;
    iters = itmax;
    for (int it = 1; it <= itmax; ++it) {
      group_rhs<GP>(L, x, v, Fv);
#pragma unroll
      for (int i = 0; i < S; ++i) t2[i] = (Fv[i] - Fn[i]) * (Fv[i] - Fn[i]);
      double d = group_sum<GP>(x, t2);
      d = sqrt(d);
      const double sprev = sig;
      sig = d / dynrm;
      if (it >= 2 && fabs(sig - sprev) <= fmax(sig, small) * 0.01) {
#pragma unroll
        for (int i = 0; i < S; ++i) v[i] = v[i] - yn[i];
        iters = it;
        break;
      }
      if (d != 0.0) {
        const double r = dynrm / d;
#pragma unroll
        for (int i = 0; i < S; ++i) v[i] = yn[i] + (Fv[i] - Fn[i]) * r;
      } else {
        const int ind = it % N;
#pragma unroll
        for (int i = 0; i < S; ++i)
          if (x.sp[i] == ind) v[i] = yn[i] - (v[i] - yn[i]);
      }
    }
    return 1.2 * sig;
  }

  // One RKC step of s stages from (yn, Fn) into y, as rkc_step.
  __device__ void step(const Grp<GP>& x, double hh, int s, double (&y)[S]) {
    const bool tab = s <= kRkcTableS;
    RkcCoef cf;
    if (!tab) cf = RkcCoef(s);
    const int row = tab ? rkc_table_row(s) - 2 : 0;
    double wjm2[S], f[S];
    const double mut1 = tab ? kRkcTable.mut1[s] : cf.mut1();
    const double mh1 = mut1 * hh;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      wjm2[i] = yn[i];
      y[i] = yn[i] + mh1 * Fn[i];
    }
    for (int j = 2; j <= s; ++j) {
      const RkcStageCoef k = tab ? kRkcTable.st[row + j] : cf.next();
      const double mh = k.mut * hh, gh = k.gt * hh;
      group_rhs<GP>(L, x, y, f);
#pragma unroll
      for (int i = 0; i < S; ++i) {
        const double wj = k.c0 * yn[i] + k.mu * y[i] + k.nu * wjm2[i] + mh * f[i] + gh * Fn[i];
        wjm2[i] = y[i];
        y[i] = wj;
      }
    }
  }

  __device__ bool attempt(const Grp<GP>& x, const Ctl& c) {
    const double hmax = c.hmax, hmin = c.hmin_rkc;
    if (attempts >= c.max_steps) {
      status = kSysMaxSteps;
      return false;
    }
    h_want = h;
    if (1.1 * h >= fabs(c.t1 - t)) h = fabs(c.t1 - t);
    if (sr_phase == 0) {
      int it;
      sigma = spec_rad(x, hmax, c.sr_itmax, it);
      ++n_sr;
      n_pow += it;
      n_rhs += it;
    }
    double y[S], F1[S], e2[S];
    if (first) {
      double hh = hmax;
      if (sigma * hh > 1.0) hh = 1.0 / sigma;
      hh = fmax(hh, hmin);
#pragma unroll
      for (int i = 0; i < S; ++i) y[i] = yn[i] + hh * Fn[i];
      group_rhs<GP>(L, x, y, F1);
      ++n_rhs;
#pragma unroll
      for (int i = 0; i < S; ++i) {
        const double est = (F1[i] - Fn[i]) / (c.atol + c.rtol * fabs(yn[i]));
        e2[i] = est * est;
      }
      const double e = group_sum<GP>(x, e2);
      const double err0 = hh * sqrt(e / (double)N);
      if (kP1 * hh < hmax * sqrt(err0))
        hh = fmax(kP1 * hh / sqrt(err0), hmin);
      else
        hh = hmax;
      h = hh;
      first = false;
    }
    const int m = rkc_stage_count(h, sigma, c.mmax);
    max_m = max(max_m, m);
    step(x, h, m, y);
    group_rhs<GP>(L, x, y, F1);
    n_rhs += m;
    ++attempts;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      double est = 0.8 * (yn[i] - y[i]) + 0.4 * h * (Fn[i] + F1[i]);
      est = est / (c.atol + c.rtol * fmax(fabs(y[i]), fabs(yn[i])));
      e2[i] = est * est;
    }
    const double err = sqrt(group_sum<GP>(x, e2) / (double)N);
    if (err > 1.0 || !crm::is_finite(err)) {
      ++n_rej;
      h = crm::is_finite(err) ? 0.8 * h / crm::pow_third_one(err) : kP1 * h;
      int it;
      sigma = spec_rad(x, hmax, c.sr_itmax, it);
      ++n_sr;
      n_pow += it;
      n_rhs += it;
      if (!(h >= hmin)) {
        status = kSysHmin;
        return false;
      }
    } else {
      cut = h < h_want;
      t += h;
      ++nstep;
      if (++sr_phase == c.sr_period) sr_phase = 0;
      ++n_acc;
      double cbrt_err, err23;
      crm::pow_third_pair(err, cbrt_err, err23);
      double fac = 10.0;
      if (!have_prev) {
        if (0.8 < fac * cbrt_err) fac = 0.8 / cbrt_err;
      } else {
        const double t1 = 0.8 * h * cbrt_err_prev;
        const double t2 = h_prev * err23;
        if (t1 < fac * t2) fac = t1 / t2;
      }
      err_prev = err;
      cbrt_err_prev = cbrt_err;
      h_prev = h;
      have_prev = true;
      gcopy<GP>(yn, y);
      gcopy<GP>(Fn, F1);
      h = h * fmax(kP1, fac);
      h = fmax(hmin, fmin(hmax, h));
      if (!group_all_finite<GP>(x, yn)) {
        status = kSysNonFinite;
        return false;
      }
    }
    return t < c.t1;
  }

  __device__ void stats(int32_t (&st)[kNStats]) const {
    st[kStAccept] = n_acc;
    st[kStReject] = n_rej;
    st[kStRhs] = n_rhs;
    st[kStSrCalls] = n_sr;
    st[kStPowIters] = n_pow;
    st[kStMaxStages] = max_m;
  }
  __device__ const double (&state() const)[S] { return yn; }
  __device__ double (&state())[S] { return yn; }
  __device__ void load_carry(const Grp<GP>& x, const Ctl& c, const double* carry, int64_t n,
                             int64_t i) {
    h = carry[(int64_t)kCarryH * n + i];
    h_prev = carry[(int64_t)kCarryHPrev * n + i];
    err_prev = carry[(int64_t)kCarryErrPrev * n + i];
    sigma = carry[(int64_t)kCarrySigma * n + i];
    nstep = (int64_t)carry[(int64_t)kCarryNstep * n + i];
    sr_phase = (int32_t)(nstep % c.sr_period);
    have_prev = carry[(int64_t)kCarryHavePrev * n + i] != 0.0;
    cbrt_err_prev = have_prev ? crm::pow_third_one(err_prev) : 0.0;
    first = false;
#pragma unroll
    for (int m = 0; m < S; ++m) {
      const int k = x.sp[m];
      v[m] = k >= 0 ? carry[(int64_t)(kCarryRows + k) * n + i] : 0.0;
    }
  }
  __device__ void store_carry(const Grp<GP>& x, double* carry, int64_t n, int64_t i) const {
#pragma unroll
    for (int m = 0; m < S; ++m) {
      const int k = x.sp[m];
      if (k >= 0) carry[(int64_t)(kCarryRows + k) * n + i] = v[m];
    }
    if (x.r != 0) return;
    carry[(int64_t)kCarryValid * n + i] = status == kSysOk ? 1.0 : 0.0;
    carry[(int64_t)kCarryH * n + i] = cut ? h_want : h;
    carry[(int64_t)kCarryHPrev * n + i] = h_prev;
    carry[(int64_t)kCarryErrPrev * n + i] = err_prev;
    carry[(int64_t)kCarrySigma * n + i] = sigma;
    carry[(int64_t)kCarryNstep * n + i] = (double)nstep;
    carry[(int64_t)kCarryHavePrev * n + i] = have_prev ? 1.0 : 0.0;
  }
};

template <class GP, int Method>
using GDriverState = typename std::conditional<Method == kMethodRkck, GRkck<GP>, GRkc<GP>>::type;

// A group's integration of one system: start / attempt / finish as Driver.
template <class GP, int Method>
struct GDriver {
  GDriverState<GP, Method> D;
  __device__ bool start(const typename GP::Params& prm, const Ctl& c, int64_t n, int64_t i,
                        const double* y0, const double* g, const Grp<GP>& x,
                        const double* carry = nullptr) {
    GP::init(D.L, prm, g, i, n, x);
    auto& y = D.state();
#pragma unroll
    for (int m = 0; m < GP::S; ++m) {
      const int k = x.sp[m];
      y[m] = k >= 0 ? y0[(int64_t)k * n + i] : 0.0;
    }
    if constexpr (Method == kMethodRkck)
      D.begin(c);
    else
      D.begin(x, c);
    if (carry && carry[(int64_t)kCarryValid * n + i] != 0.0) D.load_carry(x, c, carry, n, i);
    return D.t < c.t1;
  }
  __device__ bool attempt(const Ctl& c, const Grp<GP>& x) { return D.attempt(x, c); }
  __device__ void finish(int64_t n, int64_t i, double* y1, int32_t* status, int32_t* stats,
                         const Grp<GP>& x, double* carry = nullptr) const {
    const auto& y = D.state();
    if (carry) D.store_carry(x, carry, n, i);
    if (y1)
#pragma unroll
      for (int m = 0; m < GP::S; ++m) {
        const int k = x.sp[m];
        if (k >= 0) y1[(int64_t)k * n + i] = y[m];
      }
    if (x.r == 0) {
      int32_t st[kNStats];
      D.stats(st);
      if (status) status[i] = D.status;
      if (stats)
#pragma unroll
        for (int r = 0; r < kNStats; ++r) stats[(int64_t)r * n + i] = st[r];
    }
  }
};

template <class GP>
__device__ Grp<GP> group_of(double* lds) {
  const int lane = threadIdx.x;
  const int g = lane / GP::kL;
  const unsigned long long ones =
      GP::kL == 64 ? ~0ull : ((1ull << GP::kL) - 1ull);
  Grp<GP> x;
  x.r = lane % GP::kL;
  x.lds = lds + g * GP::kLdsPerSystem;
  x.mask = ones << (g * GP::kL);
#pragma unroll
  for (int m = 0; m < GP::S; ++m) x.sp[m] = GP::kSp[m * GP::kL + x.r];
  return x;
}

// Groups per wave and LDS doubles per wave.
template <class GP>
constexpr int kGroups = kLdsStride / GP::kL;

template <class GP>
constexpr int group_lds_doubles() {
  return kGroups<GP> * GP::kLdsPerSystem;
}

// Persistent loop at group granularity: as persistent_loop, with a group of
// kL lanes as the unit that takes a system; the refill threshold counts lanes.
template <class GP, int Method>
__device__ void group_persistent_loop(const typename GP::Params& prm, int64_t n, const double* y0,
                                      double* y1, const double* g, const Ctl& c, int32_t* status,
                                      int32_t* stats, unsigned long long* queue, double* lds,
                                      const int32_t* order, double* carry) {
  const int lane = threadIdx.x;
  const Grp<GP> x = group_of<GP>(lds);
  const int first_lane = lane - x.r;
  GDriver<GP, Method> D;
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
      if (lane == leader)
        base = atomicAdd(queue, (unsigned long long)(__popcll(need_mask) / GP::kL));
      base = __shfl(base, leader);
      if (need) {
        const unsigned long long below = need_mask & ((1ull << first_lane) - 1ull);
        const unsigned long long idx = base + (unsigned long long)(__popcll(below) / GP::kL);
        if (idx < (unsigned long long)n) {
          i = order ? (int64_t)order[idx] : (int64_t)idx;
          active = D.start(prm, c, n, i, y0, g, x, carry);
          if (!active) D.finish(n, i, y1, status, stats, x, carry);
        } else {
          retired = true;
        }
      }
    }
    if (!__ballot(!retired)) break;
    if (active && !D.attempt(c, x)) {
      D.finish(n, i, y1, status, stats, x, carry);
      active = false;
    }
  }
}

// Waves per SIMD the group kernel of a method is compiled for: a group problem
// may ask for more than the register allocator would choose by itself
// (GP::kWavesPerEuRkc, GP::kWavesPerEuRkck), spilling a few values that live
// across attempts in exchange for a second wave to hide LDS latency.
template <class GP, int Method, class = void>
struct GroupWavesPerEu {
  static constexpr int value = 1;
};
template <class GP>
struct GroupWavesPerEu<GP, kMethodRkc, std::void_t<decltype(GP::kWavesPerEuRkc)>> {
  static constexpr int value = GP::kWavesPerEuRkc;
};
template <class GP>
struct GroupWavesPerEu<GP, kMethodRkck, std::void_t<decltype(GP::kWavesPerEuRkck)>> {
  static constexpr int value = GP::kWavesPerEuRkck;
};

template <class GP, int Method, bool kPilot = false>
__global__ __launch_bounds__(kLdsStride)
__attribute__((amdgpu_waves_per_eu(GroupWavesPerEu<GP, Method>::value))) void group_persistent_kernel(
    typename GP::Params prm, int64_t n, const double* y0, double* y1,
    const double* __restrict__ g, Ctl c, int32_t* __restrict__ status,
    int32_t* __restrict__ stats, unsigned long long* queue, const int32_t* __restrict__ order,
    double* __restrict__ carry) {
  __shared__ double lds[group_lds_doubles<GP>()];
  group_persistent_loop<GP, Method>(prm, n, y0, y1, g, c, status, stats, queue, lds, order,
                                    carry);
}

template <class GP, int Method, bool kPilot>
int launch_group_method(const LaunchArgs* a, hipStream_t s) {
  const int64_t units = (a->n + kGroups<GP> - 1) / kGroups<GP>;
  if (units <= 0) return kLaunchOk;
  if (!a->ws || a->ws_bytes < kQueueBytes) return kLaunchWorkspace;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, group_persistent_kernel<GP, Method>,
                                                   kLdsStride, 0) != hipSuccess)
    return kLaunchHip;
  if (per_cu < 1) per_cu = 1;
  int64_t grid = (int64_t)cus * per_cu;
  if (grid > units) grid = units;
  unsigned long long* queue = static_cast<unsigned long long*>(a->ws);
  queue_reset_kernel<><<<1, 1, 0, s>>>(queue);
  group_persistent_kernel<GP, Method, kPilot><<<dim3((unsigned)grid), dim3(kLdsStride), 0, s>>>(
      a->prm, a->n, a->y0, a->y1, a->g, a->ctl, a->status, a->stats, queue, a->order, a->carry);
  return hipGetLastError() == hipSuccess ? kLaunchOk : kLaunchHip;
}

// Launches the one-lane kernels of Prob for the plain and persistent
// schedules and the group kernels of GP for the group schedule (the default).
template <class Prob, class GP>
int launch_with_group(const LaunchArgs* a, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (a->schedule == kSchedPlain || a->schedule == kSchedPersistent) return launch<Prob>(a, stream);
  if (!a->ws || a->ws_bytes < kQueueBytes) return launch<Prob>(a, stream);   // no queue: plain
  if (a->pilot)
    return a->method == kMethodRkck ? launch_group_method<GP, kMethodRkck, true>(a, s)
                                    : launch_group_method<GP, kMethodRkc, true>(a, s);
  return a->method == kMethodRkck ? launch_group_method<GP, kMethodRkck, false>(a, s)
                                  : launch_group_method<GP, kMethodRkc, false>(a, s);
}

template <class Prob, class GP>
int64_t workspace_with_group(int method, int schedule, int64_t n) {
  if (schedule == kSchedPlain || schedule == kSchedPersistent)
    return workspace<Prob>(method, schedule, n);
  return n > 0 ? (int64_t)kQueueBytes : 0;
}

}  // namespace rkmi
