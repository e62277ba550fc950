// rk_group.hpp -- RKCK / RKC with L lanes of a wave sharing one system.
//
// For networks whose vectors do not fit one lane's registers, a group of L
// consecutive lanes integrates one system: lane r of the group owns the
// unknowns of its slots and the rates of progress at positions p = m L + r
// (m < R), with their rate constants, all in registers.  The right-hand side
// exchanges concentrations and rates of progress through the group's LDS
// area:
//   1. owners write C_k = (rho Y_k) / W_k; [M] = sum_k C_k in species order is
//      passed along a chain of lanes (group_chain_sum) while the rates of the
//      reactions without [M] are formed;
//   2. the lane of position p writes q and -q of its reaction;
//   3. each lane sums the signed rates of its species in reaction order, then
//      f_k = (W_k omega_k) / rho,
// which is the per-system evaluation order, so results equal the one-lane
// kernels and the oracle bit for bit.  Weighted norms (sums in species order)
// take the same chain, so the step-size controller runs identically (and
// redundantly) in the L lanes.  The groups of a wave hold different systems
// and may diverge like lanes do.
//
// A group problem GP supplies N, NR, kL (lanes per system), S (= 2 slots), R,
// kMSlot (the first slot whose reactions may have a one-species side times
// [M]), the LDS layout (kOffC, kOffQ, kSentinel, kNegOff, kOffRed,
// kLdsPerSystem: +q at kOffQ + p, the zero at kOffQ + kSentinel, -q at
// kOffQ + kNegOff + p), the tables kSp (species of slot m of lane r at
// m L + r, -1 for none), kRx (packed operand species of each position's
// reaction, [M] as index N; lane-major, kRxWords per lane), kTc (each lane's
// signed rate positions, packed, lane-major, kTcWords per lane:
// its slot-0 species' list padded with the zero to whole chunks of kChunk
// terms, then its slot-1 species' list, kTermLen in all), kBnd (the chunks
// of the slot-0 list) and kSwitchChunks (the chunks at whose end some lane
// switches), Params, Lane, init(Lane&, prm, g, i, n, x).
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
// The same for a double: the value is formed here, not later.
__device__ inline void opaque_f64(double& v) { asm volatile("" : "+v"(v)); }

template <class GP>
__device__ inline bool owns(const Grp<GP>& x, int m) {
  return x.sp[m] >= 0;
}

// v shifted one lane up within each row of 16 lanes (lane i gets lane i - 1's
// value; the first lane of a row gets +0).
__device__ inline double dpp_row_shr1(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x111, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x111, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// ((0 + v_0) + v_1) + ... + v_{n-1}: the sum of n values of the group's LDS
// area at v (16-byte aligned) in index order, returned to every lane of the
// group.  Lane r of the group takes v_{8r} .. v_{8r+7}; the running sum passes
// from lane to lane (lane r adds its values, in order, to the sum of the lanes
// before it), so each addition is the one of the serial loop.  Adding +0 for
// the slots past n changes nothing: a sum that starts at +0 is never -0.  The
// chain stays within one row of 16 lanes (a group starts at a multiple of kL).
// The same chain one lane step at a time (step() kLanes times, then
// result()), so that independent work can be placed between the steps.
template <class GP, int Nv>
struct ChainSum {
  static constexpr int kPer = 8, kLanes = (Nv + kPer - 1) / kPer;
  static_assert(kLanes <= GP::kL && kLanes <= 16, "chain within a row of the group");
  double a[kPer];
  double s;
  int r;
  __device__ ChainSum(const Grp<GP>& x, const double* v) : s(0.0), r(x.r) {
    const double2* p = reinterpret_cast<const double2*>(v + (r < kLanes ? kPer * r : 0));
#pragma unroll
    for (int q = 0; q < kPer / 2; ++q) {
      const double2 u = p[q];
      a[2 * q] = u.x;
      a[2 * q + 1] = u.y;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q)
      if (kPer * (kLanes - 1) + q >= Nv) a[q] = (r == kLanes - 1) ? 0.0 : a[q];
  }
  __device__ void step() {
    double u = dpp_row_shr1(s);
    if (GP::kL < 16) u = r == 0 ? 0.0 : u;
#pragma unroll
    for (int q = 0; q < kPer; ++q) u = u + a[q];
    s = u;
  }
  __device__ double result() const { return __shfl(s, kLanes - 1, GP::kL); }
};

template <class GP, int Nv>
__device__ double group_chain_sum(const Grp<GP>& x, const double* v) {
  ChainSum<GP, Nv> ch(x, v);
#pragma unroll
  for (int step = 0; step < ChainSum<GP, Nv>::kLanes; ++step) ch.step();
  return ch.result();
}

// Two such sums in one pass along the chain (the values of u and w in index
// order, each from +0), both returned to every lane of the group.
template <class GP, int Nv>
__device__ void group_chain_sum2(const Grp<GP>& x, const double* u, const double* w, double& su,
                                 double& sw) {
  constexpr int kPer = 8, kLanes = (Nv + kPer - 1) / kPer;
  static_assert(kLanes <= GP::kL && kLanes <= 16, "chain within a row of the group");
  const int r = x.r;
  const int off = r < kLanes ? kPer * r : 0;
  const double2* pu = reinterpret_cast<const double2*>(u + off);
  const double2* pw = reinterpret_cast<const double2*>(w + off);
  double a[kPer], b[kPer];
#pragma unroll
  for (int q = 0; q < kPer / 2; ++q) {
    const double2 s = pu[q], t = pw[q];
    a[2 * q] = s.x;
    a[2 * q + 1] = s.y;
    b[2 * q] = t.x;
    b[2 * q + 1] = t.y;
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q)
    if (kPer * (kLanes - 1) + q >= Nv) {
      a[q] = (r == kLanes - 1) ? 0.0 : a[q];
      b[q] = (r == kLanes - 1) ? 0.0 : b[q];
    }
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int step = 0; step < kLanes; ++step) {
    double v1 = dpp_row_shr1(s1), v2 = dpp_row_shr1(s2);
    if (GP::kL < 16) {
      v1 = r == 0 ? 0.0 : v1;
      v2 = r == 0 ? 0.0 : v2;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      v1 = v1 + a[q];
      v2 = v2 + b[q];
    }
    s1 = v1;
    s2 = v2;
  }
  su = __shfl(s1, kLanes - 1, GP::kL);
  sw = __shfl(s2, kLanes - 1, GP::kL);
}

// sum_k t_k over k = 0..N-1 in order, t_k held by the owners; every lane of
// the group gets the same value.
template <class GP>
__device__ double group_sum(const Grp<GP>& x, const double (&t)[GP::S]) {
  double* red = x.lds + GP::kOffRed;
#pragma unroll
  for (int m = 0; m < GP::S; ++m)
    if (owns<GP>(x, m)) red[x.sp[m]] = t[m];
  group_sync();
  const double s = group_chain_sum<GP, GP::N>(x, red);
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

// A group problem with the energy equation (GP::kThermal: unknowns T, Y).
template <class GP, class = void>
struct GroupThermal {
  static constexpr bool value = false;
};
template <class GP>
struct GroupThermal<GP, std::void_t<decltype(GP::kThermal)>> {
  static constexpr bool value = GP::kThermal;
};

template <class GP>
__device__ void group_rhs_mass_action(const typename GP::Lane& L, const Grp<GP>& x,
                                      const double (&y)[GP::S], double (&f)[GP::S]);
template <class GP>
__device__ void group_rhs_thermal(const typename GP::Lane& L, const Grp<GP>& x,
                                  const double (&y)[GP::S], double (&f)[GP::S]);

// Right-hand side of the group's system at y (owned slots) into f.
template <class GP>
__device__ void group_rhs(const typename GP::Lane& L, const Grp<GP>& x, const double (&y)[GP::S],
                          double (&f)[GP::S]) {
  if constexpr (GroupOwnRhs<GP>::value)
    GP::rhs(L, x, y, f);
  else if constexpr (GroupThermal<GP>::value)
    group_rhs_thermal<GP>(L, x, y, f);
  else
    group_rhs_mass_action<GP>(L, x, y, f);
}

// Lane r's row of a lane-major code table (Words 32-bit words, a multiple of
// four, 16-byte aligned) as whole-vector loads.
template <int Words>
__device__ inline void load_row(const uint32_t* table, int row, uint32_t (&w)[Words]) {
  static_assert(Words % 4 == 0, "rows of whole 16-byte vectors");
  const uint4* const v = reinterpret_cast<const uint4*>(table) + row * (Words / 4);
#pragma unroll
  for (int q = 0; q < Words / 4; ++q) {
    const uint4 u = v[q];
    w[4 * q] = u.x;
    w[4 * q + 1] = u.y;
    w[4 * q + 2] = u.z;
    w[4 * q + 3] = u.w;
  }
}

// Mass action: concentrations, [M] and rates of progress exchanged through
// the group's LDS area (the scheme in the header comment).
template <class GP>
__device__ void group_rhs_mass_action(const typename GP::Lane& L, const Grp<GP>& x,
                                      const double (&y)[GP::S], double (&f)[GP::S]) {
  static_assert(GP::S == 2 && GP::kOffC % 2 == 0, "two species slots per lane, aligned C");
  static_assert(GP::kOffC + GP::N < GP::kOffQ && GP::kSentinel == GP::R * GP::kL &&
                    GP::kOffQ + GP::kSentinel < GP::kOffRed &&
                    GP::kOffRed + GP::N <= GP::kOffQ + GP::kNegOff &&
                    GP::kOffQ + GP::kNegOff + GP::R * GP::kL <= GP::kLdsPerSystem,
                "C, +q, the zero, the scratch and -q are disjoint");
  constexpr int N = GP::N, LL = GP::kL;
  double* const C = x.lds + GP::kOffC;
  double* const Q = x.lds + GP::kOffQ;
  // the operand and term tables are read from constant memory at each
  // evaluation (vector loads, cached, issued here so that the exchanges below
  // cover their latency), not held in registers across the integration
  const int row = opaque_zero() + x.r;
  uint32_t rxw[GP::kRxWords];
  load_row<GP::kRxWords>(GP::kRx, row, rxw);
#pragma unroll
  for (int m = 0; m < GP::S; ++m)
    if (owns<GP>(x, m)) C[x.sp[m]] = (L.rho * y[m]) * L.iW[m];
  group_sync();
  // [M] by the chain of lanes, its steps interleaved with the rates of the
  // slots before the first one that needs [M] (they hide the chain's
  // dependent additions)
  ChainSum<GP, N> chain(x, C);
  constexpr int kChainSteps = ChainSum<GP, N>::kLanes;
  static_assert(kChainSteps <= GP::kMSlot || GP::kMSlot == GP::R, "[M] formed before its slots");
  double M = 0.0;
  uint32_t tcw[GP::kTcWords];
#pragma unroll
  for (int m = 0; m < GP::R; ++m) {
    if (m < kChainSteps) chain.step();
    if (m == kChainSteps - 1) {
      M = chain.result();
      load_row<GP::kTcWords>(GP::kTc, row, tcw);
    }
    const int p = m * LL + x.r;
    const uint32_t code = rxw[m];
    const uint32_t ib = (code >> 8) & 0xffu, id = code >> 24;
    const double ca = C[code & 0xffu], cc = C[(code >> 16) & 0xffu];
    double cb = C[ib], cd = C[id];
    if (m >= GP::kMSlot) {
      // a one-species side: its second factor is [M]
      cb = ib == (uint32_t)N ? M : cb;
      cd = id == (uint32_t)N ? M : cd;
    }
    const double q = (L.kf[m] * ca) * cb - (L.kr[m] * cc) * cd;
    Q[p] = q;
    Q[GP::kNegOff + p] = -q;
    // bound how far the scheduler moves loads ahead (register pressure)
    if (m % 2 == 1) __builtin_amdgcn_sched_barrier(0);
  }
  group_sync();
  // each lane's signed rates: its slot-0 species' terms (padded to whole
  // chunks with the zero), then from chunk L.bnd on its slot-1 species'; the
  // accumulator moves to slot 0 at the end of chunk L.bnd - 1
  double acc = 0.0, om0 = 0.0;
#pragma unroll
  for (int t = 0; t < GP::kTermLen; ++t) {
    // term t: kTermBits-bit position in the signed rates, packed
    // kTermsPerWord to a register; om - q is formed as om + (-q)
    const uint32_t word = tcw[t / GP::kTermsPerWord];
    const uint32_t code = (word >> ((t % GP::kTermsPerWord) * GP::kTermBits)) &
                          ((1u << GP::kTermBits) - 1u);
    acc = acc + Q[code];
    if (t % GP::kChunk == GP::kChunk - 1 && ((GP::kSwitchChunks >> (t / GP::kChunk)) & 1)) {
      const bool sw = t / GP::kChunk + 1 == L.bnd;
      om0 = sw ? acc : om0;
      acc = sw ? 0.0 : acc;
    }
    if (t % 16 == 15) {
      // keep the additions near their loads (else all loads are issued first
      // and held in registers; sixteen in flight: 6 % over four)
      opaque_f64(acc);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  f[0] = owns<GP>(x, 0) ? (L.W[0] * om0) * L.irho : 0.0;
  f[1] = owns<GP>(x, 1) ? (L.W[1] * acc) * L.irho : 0.0;
}

// Mass action with the energy equation (Sec. 4.2 at constant volume): the
// owner of T writes it beside the concentrations, every lane reads it and
// forms ln T and 1/T, each position's lane its reaction's rate coefficients
// k_f = exp(ln A + b ln T - E (1/T)) and k_r = k_f (1/K) (read from the
// uniform data at every evaluation), the species part as
// group_rhs_mass_action, then the species owners write (e_k omega_k) W_k and
// Y_k c_v,k(T) and two chain sums over the species give
// dT/dt = -((sum * (1/rho)) / c_v): the reference evaluation's operations in
// its order.
template <class GP>
__device__ void group_rhs_thermal(const typename GP::Lane& L, const Grp<GP>& x,
                                  const double (&y)[GP::S], double (&f)[GP::S]) {
  static_assert(GP::S == 2 && GP::kOffC % 2 == 0 && GP::kOffE1 % 2 == 0 && GP::kOffE2 % 2 == 0,
                "two unknowns per lane, aligned areas");
  static_assert(sizeof(RkcCoef) <= sizeof(double) * (GP::kOffE1 - GP::kOffRed),
                "the energy rows leave the RKC coefficients kept in the scratch intact");
  static_assert(GP::kOffC + GP::NS < GP::kOffT && GP::kOffT < GP::kOffQ &&
                    GP::kSentinel == GP::R * GP::kL && GP::kOffQ + GP::kSentinel < GP::kOffRed &&
                    GP::kOffRed + GP::N <= GP::kOffQ + GP::kNegOff &&
                    GP::kOffE1 + GP::NS <= GP::kOffE2 &&
                    GP::kOffE2 + GP::NS <= GP::kOffQ + GP::kNegOff &&
                    GP::kOffQ + GP::kNegOff + GP::R * GP::kL <= GP::kLdsPerSystem,
                "C, T, +q, the zero, the scratch, the energy rows and -q are disjoint");
  constexpr int NS = GP::NS, NR = GP::NR, LL = GP::kL;
  const double* const p = L.prm;
  double* const C = x.lds + GP::kOffC;
  double* const Q = x.lds + GP::kOffQ;
  const int z0 = opaque_zero();
  const uint32_t* const rxl = GP::kRx + (z0 + x.r) * GP::kRxWords;
#pragma unroll
  for (int m = 0; m < GP::S; ++m) {
    const int u = x.sp[m];
    if (u == 0) x.lds[GP::kOffT] = y[m];
    if (u > 0) C[u - 1] = (L.rho * y[m]) * L.iW[m];
  }
  group_sync();
  const double T = x.lds[GP::kOffT];
  const double lnT = crm::cr_log(T);
  const double invT = 1.0 / T;
  const double M = group_chain_sum<GP, NS>(x, C);
  uint32_t tcw[GP::kTcWords];
  load_row<GP::kTcWords>(GP::kTc, z0 + x.r, tcw);
  // two slots per iteration: their exponentials' table reads overlap (2.3 %
  // over a rolled loop at 53 species)
#pragma unroll 2
  for (int m = 0; m < GP::R; ++m) {
    const int pos = m * LL + x.r;
    const int j = GP::kRxOf[pos + z0];
    double kf = 0.0, kr = 0.0;
    if (j >= 0) {
      kf = crm::cr_exp(p[j] + p[NR + j] * lnT - p[2 * NR + j] * invT);
      kr = kf * p[3 * NR + j];
    }
    const uint32_t code = rxl[m];
    const uint32_t ib = (code >> 8) & 0xffu, id = code >> 24;
    const double ca = C[code & 0xffu], cc = C[(code >> 16) & 0xffu];
    double cb = C[ib], cd = C[id];
    if (m >= GP::kMSlot) {
      cb = ib == (uint32_t)NS ? M : cb;
      cd = id == (uint32_t)NS ? M : cd;
    }
    const double q = (kf * ca) * cb - (kr * cc) * cd;
    Q[pos] = q;
    Q[GP::kNegOff + pos] = -q;
  }
  group_sync();
  double acc = 0.0, om0 = 0.0;
#pragma unroll
  for (int t = 0; t < GP::kTermLen; ++t) {
    uint32_t word = tcw[t / GP::kTermsPerWord];
    opaque(word);
    const uint32_t code = (word >> ((t % GP::kTermsPerWord) * GP::kTermBits)) &
                          ((1u << GP::kTermBits) - 1u);
    acc = acc + Q[code];
    if (t % GP::kChunk == GP::kChunk - 1 && ((GP::kSwitchChunks >> (t / GP::kChunk)) & 1)) {
      const bool sw = t / GP::kChunk + 1 == L.bnd;
      om0 = sw ? acc : om0;
      acc = sw ? 0.0 : acc;
    }
    if (t % 4 == 3) {
      opaque_f64(acc);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  const double om[2] = {om0, acc};
  // the energy sums' terms, species by species
  double* const R1 = x.lds + GP::kOffE1;
  double* const R2 = x.lds + GP::kOffE2;
#pragma unroll
  for (int m = 0; m < GP::S; ++m) {
    const int u = x.sp[m];
    f[m] = u > 0 ? (L.W[m] * om[m]) * L.irho : 0.0;
    if (u > 0) {
      const double e = L.u0[m] + (L.cv0[m] + L.cv1[m] * T) * T;
      R1[u - 1] = (e * om[m]) * L.W[m];
      R2[u - 1] = y[m] * (L.cv0[m] + 2.0 * L.cv1[m] * T);
    }
  }
  group_sync();
  double sum, cv;
  group_chain_sum2<GP, NS>(x, R1, R2, sum, cv);
  group_sync();
#pragma unroll
  for (int m = 0; m < GP::S; ++m)
    if (x.sp[m] == 0) f[m] = -((sum * L.irho) / cv);
}

template <class GP>
__device__ void gcopy(double (&d)[GP::S], const double (&s)[GP::S]) {
#pragma unroll
  for (int m = 0; m < GP::S; ++m) d[m] = s[m];
}

// The group RKC driver is a state machine at right-hand-side granularity: it
// always holds the argument z of its next evaluation, and advance() consumes
// the value f(z), runs the method's arithmetic up to the next evaluation it
// needs (or the end of the integration) and sets z again.  The persistent
// loop evaluates every active group's f(z) at one place, so the groups of a
// wave evaluate together whatever step, stage count or power iteration each
// is in, and a group that finishes takes a new system at the next evaluation.
// RKCK attempts always take the same six evaluations, so its group driver
// runs attempt by attempt (GRkckAttempt, group_attempt_loop).  The operations
// and their order are those of the one-lane drivers (rk_device.hpp), hence
// the same bits.

// -------------------------------------------------------------------- RKC
template <class GP>
struct GRkc {
  static constexpr int S = GP::S, N = GP::N;
  enum : int32_t { kPhBegin, kPhPower, kPhFirst, kPhStage, kPhError };
  typename GP::Lane L;
  double yn[S], Fn[S], v[S], y[S], w2[S], z[S];
  double t, h, h_prev, err_prev, sigma, cbrt_err_prev, h_want;
  double hh;            // the first step's trial size
  double p_sig, p_dyn;  // power method: last estimate, perturbation size
  int64_t nstep, attempts;
  int32_t sr_phase;     // nstep mod sr_period
  int32_t p_it;         // power method: iteration of the pending evaluation
  int32_t st_j, st_m;   // stage j of m of the pending evaluation
  int32_t phase;
  int32_t n_acc, n_rej, n_rhs, n_sr, n_pow, max_m, status;
  bool first, have_prev, cut, p_rejected, v_carried;

  __device__ bool begin(const Grp<GP>& x, const Ctl& c) {
    t = c.t0;
    status = kSysOk;
    attempts = 0;
    n_acc = n_rej = n_rhs = n_sr = n_pow = max_m = 0;
    h = h_prev = err_prev = sigma = cbrt_err_prev = h_want = 0.0;
    nstep = 0;
    sr_phase = 0;
    first = true;
    have_prev = false;
    cut = false;
    v_carried = false;
    if (t < c.t1) {
      gcopy<GP>(z, yn);
      phase = kPhBegin;
      return true;
    }
#pragma unroll
    for (int i = 0; i < S; ++i) Fn[i] = v[i] = 0.0;
    return false;
  }

  // Nonlinear power method (Appendix), as spec_rad: the set-up up to the
  // first evaluation f(v).
  __device__ void power_start(const Grp<GP>& x, bool after_reject) {
    double t2[S];
    const double sq = sqrt(kUround);
#pragma unroll
    for (int i = 0; i < S; ++i) t2[i] = yn[i] * yn[i];
    double ynrm = group_sum<GP>(x, t2);
#pragma unroll
    for (int i = 0; i < S; ++i) t2[i] = v[i] * v[i];
    double vnrm = group_sum<GP>(x, t2);
    ynrm = sqrt(ynrm);
    vnrm = sqrt(vnrm);
    if (ynrm != 0.0 && vnrm != 0.0) {
      p_dyn = ynrm * sq;
      const double r = p_dyn / vnrm;
#pragma unroll
      for (int i = 0; i < S; ++i) v[i] = yn[i] + v[i] * r;
    } else if (ynrm != 0.0) {
      p_dyn = ynrm * sq;
#pragma unroll
      for (int i = 0; i < S; ++i) v[i] = yn[i] * (1.0 + sq);
    } else if (vnrm != 0.0) {
      p_dyn = kUround;
      const double r = p_dyn / vnrm;
#pragma unroll
      for (int i = 0; i < S; ++i) v[i] = v[i] * r;
    } else {
      p_dyn = kUround;
#pragma unroll
      for (int i = 0; i < S; ++i) v[i] = owns<GP>(x, i) ? kUround : 0.0;
    }
    p_sig = 0.0;
    p_it = 1;
    p_rejected = after_reject;
    gcopy<GP>(z, v);
    phase = kPhPower;
  }

  // One power iteration on Fv = f(v); true when the estimate is final.
  __device__ bool power_step(const Grp<GP>& x, const Ctl& c, const double (&Fv)[S]) {
    double t2[S];
    ++n_rhs;
#pragma unroll
    for (int i = 0; i < S; ++i) t2[i] = (Fv[i] - Fn[i]) * (Fv[i] - Fn[i]);
    double d = group_sum<GP>(x, t2);
    d = sqrt(d);
    const double sprev = p_sig;
    p_sig = d / p_dyn;
    const double small = 1.0 / c.hmax;
    if (p_it >= 2 && fabs(p_sig - sprev) <= fmax(p_sig, small) * 0.01) {
#pragma unroll
      for (int i = 0; i < S; ++i) v[i] = v[i] - yn[i];
      n_pow += p_it;
      return true;
    }
    if (d != 0.0) {
      const double r = p_dyn / d;
#pragma unroll
      for (int i = 0; i < S; ++i) v[i] = yn[i] + (Fv[i] - Fn[i]) * r;
    } else {
      const int ind = p_it % N;
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (x.sp[i] == ind) v[i] = yn[i] - (v[i] - yn[i]);
    }
    if (p_it >= c.sr_itmax) {
      n_pow += c.sr_itmax;
      return true;
    }
    ++p_it;
    gcopy<GP>(z, v);
    return false;
  }

  // Coefficients of stage j of an s-stage step: tabulated, or the recurrence
  // (RkcCoef) kept in the group's norm scratch between evaluations.
  __device__ RkcStageCoef stage_coef(const Grp<GP>& x, int s, int j) {
    if (s <= kRkcTableS) return kRkcTable.st[rkc_table_row(s) + j - 2];
    static_assert(sizeof(RkcCoef) <= sizeof(double) * GP::N, "recurrence fits the scratch");
    RkcCoef* keep = reinterpret_cast<RkcCoef*>(x.lds + GP::kOffRed);
    RkcCoef cf = *keep;
    const RkcStageCoef k = cf.next();
    group_sync();
    if (x.r == 0) *keep = cf;
    group_sync();
    return k;
  }

  // The attempt from its start (after an accepted step, a rejection's power
  // method, or the first evaluation) up to its first evaluation.
  __device__ bool next_attempt(const Grp<GP>& x, const Ctl& c) {
    if (!(t < c.t1)) return false;
    if (attempts >= c.max_steps) {
      status = kSysMaxSteps;
      return false;
    }
    h_want = h;
    if (1.1 * h >= fabs(c.t1 - t)) h = fabs(c.t1 - t);
    if (sr_phase == 0) {
      power_start(x, false);
      return true;
    }
    return after_power(x, c);
  }

  // The attempt after its spectral radius: the first step's trial evaluation,
  // or the stages.
  __device__ bool after_power(const Grp<GP>& x, const Ctl& c) {
    if (first) {
      hh = c.hmax;
      if (sigma * hh > 1.0) hh = 1.0 / sigma;
      hh = fmax(hh, c.hmin_rkc);
#pragma unroll
      for (int i = 0; i < S; ++i) z[i] = yn[i] + hh * Fn[i];
      phase = kPhFirst;
      return true;
    }
    return start_stages(x, c);
  }

  __device__ bool start_stages(const Grp<GP>& x, const Ctl& c) {
    st_m = rkc_stage_count(h, sigma, c.mmax);
    max_m = max(max_m, st_m);
    double mut1;
    if (st_m <= kRkcTableS) {
      mut1 = kRkcTable.mut1[st_m];
    } else {
      const RkcCoef cf(st_m);
      mut1 = cf.mut1();
      group_sync();
      if (x.r == 0) *reinterpret_cast<RkcCoef*>(x.lds + GP::kOffRed) = cf;
      group_sync();
    }
    const double mh1 = mut1 * h;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      w2[i] = yn[i];
      y[i] = yn[i] + mh1 * Fn[i];
    }
    st_j = 2;
    gcopy<GP>(z, y);
    phase = kPhStage;
    return true;
  }

  // Consumes f(z); false when the integration has ended.
  __device__ bool advance(const Grp<GP>& x, const Ctl& c, const double (&f)[S]) {
    switch (phase) {
      case kPhBegin:
        gcopy<GP>(Fn, f);
        ++n_rhs;
        if (!v_carried) gcopy<GP>(v, Fn);
        return next_attempt(x, c);
      case kPhPower:
        if (!power_step(x, c, f)) return true;
        sigma = 1.2 * p_sig;
        ++n_sr;
        if (p_rejected) {
          if (!(h >= c.hmin_rkc)) {
            status = kSysHmin;
            return false;
          }
          return next_attempt(x, c);
        }
        return after_power(x, c);
      case kPhFirst: {
        ++n_rhs;
        double e2[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
          const double est = (f[i] - Fn[i]) / (c.atol + c.rtol * fabs(yn[i]));
          e2[i] = est * est;
        }
        const double e = group_sum<GP>(x, e2);
        const double err0 = hh * sqrt(e / (double)N);
        if (kP1 * hh < c.hmax * sqrt(err0))
          hh = fmax(kP1 * hh / sqrt(err0), c.hmin_rkc);
        else
          hh = c.hmax;
        h = hh;
        first = false;
        return start_stages(x, c);
      }
      case kPhStage: {
        const RkcStageCoef k = stage_coef(x, st_m, st_j);
        const double mh = k.mut * h, gh = k.gt * h;
#pragma unroll
        for (int i = 0; i < S; ++i) {
          const double wj = k.c0 * yn[i] + k.mu * y[i] + k.nu * w2[i] + mh * f[i] + gh * Fn[i];
          w2[i] = y[i];
          y[i] = wj;
        }
        if (++st_j > st_m) phase = kPhError;
        gcopy<GP>(z, y);
        return true;
      }
      default:
        break;
    }
    // kPhError: f = f(w_s), the error estimate and the controller
    n_rhs += st_m;
    ++attempts;
    double e2[S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
      double est = 0.8 * (yn[i] - y[i]) + 0.4 * h * (Fn[i] + f[i]);
      est = est / (c.atol + c.rtol * fmax(fabs(y[i]), fabs(yn[i])));
      e2[i] = est * est;
    }
    const double err = sqrt(group_sum<GP>(x, e2) / (double)N);
    if (err > 1.0 || !crm::is_finite(err)) {
      ++n_rej;
      h = crm::is_finite(err) ? 0.8 * h / crm::pow_third_one(err) : kP1 * h;
      power_start(x, true);
      return true;
    }
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
    gcopy<GP>(Fn, f);
    h = h * fmax(kP1, fac);
    h = fmax(c.hmin_rkc, fmin(c.hmax, h));
    if (!group_all_finite<GP>(x, yn)) {
      status = kSysNonFinite;
      return false;
    }
    return next_attempt(x, c);
  }

  // The next advance runs the error estimate and the controller.
  __device__ bool at_error() const { return phase == kPhError; }
  // Evaluations before that while in the stages (else 0).
  __device__ int to_error() const { return phase == kPhStage ? st_m - st_j + 1 : 0; }

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
  // carried controller state, applied before the first evaluation f(t0, y0)
  __device__ bool load_carry(const Grp<GP>& x, const Ctl& c, const double* carry, int64_t n,
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
    v_carried = true;
    return true;   // the pending evaluation f(t0, y0) stays
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
using GDriverState = GRkc<GP>;

// A group's integration of one system: start (true while an evaluation is
// pending), advance (consumes f(z)), finish.
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
    bool pending = D.begin(x, c);
    if (pending && carry && carry[(int64_t)kCarryValid * n + i] != 0.0)
      pending = D.load_carry(x, c, carry, n, i);
    return pending;
  }
  __device__ const double (&arg() const)[GP::S] { return D.z; }
  __device__ bool advance(const Ctl& c, const Grp<GP>& x, const double (&f)[GP::S]) {
    return D.advance(x, c, f);
  }
  __device__ bool at_error() const { return D.at_error(); }
  __device__ int to_error() const { return D.to_error(); }
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
  static_assert(GP::kLdsPerSystem % 2 == 0 && GP::kOffRed % 2 == 0,
                "16-byte aligned group areas (chain sums read pairs)");
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

// Group RKCK attempt by attempt: all six evaluations of an attempt in one
// straight sequence, the groups of a wave refilled between attempts.  Every
// attempt takes the same evaluations, so the groups of a wave stay in step
// and an evaluation-granular state machine only adds its dispatch (53
// species at 2^16 systems: 863 against 1009 ms; Pleiades, eight groups per
// wave, 19.6 against 34.4 ms).
// RKCK by attempts: the arithmetic of the one-lane driver, in its order.
template <class GP>
struct GRkckAttempt {
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

  // One attempt; false when the integration has ended.
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
};

// The attempt-granular loop for such problems: a group takes a system, runs
// attempts until it ends, and the wave refills idle groups between attempts.
template <class GP>
__device__ void group_attempt_finish(const GRkckAttempt<GP>& D, const Grp<GP>& x, int64_t n,
                                     int64_t i, double* y1, int32_t* status, int32_t* stats,
                                     double* carry) {
  if (carry && x.r == 0) {
    carry[(int64_t)kCarryValid * n + i] = D.status == kSysOk ? 1.0 : 0.0;
    carry[(int64_t)kCarryH * n + i] = D.cut ? D.h_want : D.h;
  }
  if (y1)
#pragma unroll
    for (int m = 0; m < GP::S; ++m) {
      const int k = x.sp[m];
      if (k >= 0) y1[(int64_t)k * n + i] = D.y[m];
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

template <class GP>
__device__ void group_attempt_loop(const typename GP::Params& prm, int64_t n, const double* y0,
                                   double* y1, const double* g, const Ctl& c, int32_t* status,
                                   int32_t* stats, unsigned long long* queue, double* lds,
                                   const int32_t* order, double* carry) {
  const int lane = threadIdx.x;
  const Grp<GP> x = group_of<GP>(lds);
  const int first_lane = lane - x.r;
  GRkckAttempt<GP> D;
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
          GP::init(D.L, prm, g, i, n, x);
#pragma unroll
          for (int m = 0; m < GP::S; ++m) {
            const int k = x.sp[m];
            D.y[m] = k >= 0 ? y0[(int64_t)k * n + i] : 0.0;
          }
          D.begin(c);
          active = D.t < c.t1;
          // the carried step applies to an integration that has a step to take
          if (active && carry && carry[(int64_t)kCarryValid * n + i] != 0.0) {
            D.h = carry[(int64_t)kCarryH * n + i];
            D.h_want = D.h;
          }
          if (!active) group_attempt_finish<GP>(D, x, n, i, y1, status, stats, carry);
        } else {
          retired = true;
        }
      }
    }
    if (!__ballot(!retired)) break;
    if (active && !D.attempt(x, c)) {
      group_attempt_finish<GP>(D, x, n, i, y1, status, stats, carry);
      active = false;
    }
  }
}

// Default of Ctl::align (the RKC state machine; RKCK groups run whole
// attempts and stay in step): on the 53-species network at 2^16 systems the
// RKC kernel took 760 / 742 / 753 / 767 ms with no waiting / 1 / 2 / 5 (32
// species, four groups per wave: 505 / 472 / 525 / 590 ms with none / 1 / 3 /
// 8).  With
// the energy equation the evaluation (an exponential per reaction) outweighs
// the controller, and waiting costs more than it saves (53 species + T at
// 2^18 systems: 8.54 s without, 8.71 s with 1).
template <class GP, int Method>
constexpr int group_align_default() {
  return GroupThermal<GP>::value ? 0 : 1;
}

// Persistent loop at group granularity: as persistent_loop, with a group of
// kL lanes as the unit that takes a system and one right-hand-side
// evaluation as the unit of progress; the refill threshold counts lanes.
template <class GP, int Method>
__device__ void group_persistent_loop(const typename GP::Params& prm, int64_t n, const double* y0,
                                      double* y1, const double* g, const Ctl& c, int32_t* status,
                                      int32_t* stats, unsigned long long* queue, double* lds,
                                      const int32_t* order, double* carry) {
  if constexpr (Method == kMethodRkck) {
    group_attempt_loop<GP>(prm, n, y0, y1, g, c, status, stats, queue, lds, order, carry);
    return;
  }
  const int lane = threadIdx.x;
  const Grp<GP> x = group_of<GP>(lds);
  const int first_lane = lane - x.r;
  GDriver<GP, Method> D;
  int64_t i = -1;
  bool active = false, retired = false;
  const int align = c.align > 0 ? c.align : (c.align == 0 ? group_align_default<GP, Method>() : 0);
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
    // Phase alignment: the groups of a wave evaluate together, but the code
    // that follows an evaluation depends on each group's phase, and groups in
    // different phases run their codes one after the other.  A group whose
    // next step is the error estimate and the controller (the longest of
    // them) waits while another group is at most `align` evaluations from
    // its own, so that both run it together; its arithmetic is unchanged.
    bool run = active;
    if (align > 0) {
      const int te = active ? D.to_error() : 0;
      if (__ballot(te > 0 && te <= align) && active && D.at_error()) run = false;
    }
    if (run) {
      double f[GP::S];
      group_rhs<GP>(D.D.L, x, D.arg(), f);
      if (!D.advance(c, x, f)) {
        D.finish(n, i, y1, status, stats, x, carry);
        active = false;
      }
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
  __shared__ __attribute__((aligned(16))) double lds[group_lds_doubles<GP>()];
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

// Launches the group kernels of GP under every schedule (problems without
// one-lane kernels).
template <class GP>
int launch_group_only(const LaunchArgs* a, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (a->n > 0 && (!a->ws || a->ws_bytes < kQueueBytes)) return kLaunchWorkspace;
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
