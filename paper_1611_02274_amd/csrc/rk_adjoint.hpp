// rk_adjoint.hpp -- discrete adjoints of the RKC and RKCK step sequences.
//
// The gradient is that of the map from y(t0) (and the problem's parameters
// theta) to y(t1) through the accepted steps, with each step's size h_k and
// stage count s_k held at the values the controller chose (rejected attempts,
// the controller and the spectral-radius estimates are not differentiated).
// Sec. 2.2 stage recursion, transposed: for a loss L with lambda = dL/dy(t1),
//   for j = s..2:  w0^ += (1 - mu_j - nu_j) wj^,  w_{j-1}^ += mu_j wj^,
//                  w_{j-2}^ += nu_j wj^,  F0^ += gt_j h wj^,
//                  u = mut_j h wj^:  w_{j-1}^ += J(w_{j-1})^T u,
//                  theta^ += (df/dtheta)(w_{j-1})^T u;
//   w0^ += w1^,  F0^ += mut_1 h w1^,  w0^ += J(w_0)^T F0^,
//   theta^ += (df/dtheta)(w_0)^T F0^,  and lambda = w0^ for the step before.
//
// Forward: the ordinary RKC integration, recording every accepted step's
// (h, s) and the state every K accepted steps (the tape).  Reverse: per
// segment of K steps, last segment first, the step-start states are
// recomputed from the segment's checkpoint; per step, last first, the stages
// w_0..w_{s-1} and their coefficients are recomputed into the lane's columns
// and the transposed recursion runs in registers.  One lane per system.
//
// RKCK (Sec. 2.1 stage equations with the Table 1 coefficients), step sizes
// held fixed: with z_1 = y, z_i = y + sum_{j<i} b_ij k_j, k_i = h f(z_i) and
// y' = y + sum_i c_i k_i, the transpose for lambda = dL/dy' is
//   kbar_i = c_i lambda,  ybar = lambda;  for i = 6..1:
//     u = h kbar_i,  zbar = J(z_i)^T u,  theta^ += (df/dtheta)(z_i)^T u,
//     ybar += zbar,  kbar_j += b_ij zbar (j < i);
// ybar is lambda for the step before.  The reverse sweep recomputes a step's
// stage arguments z_i into the lane's columns, next to the zbar_i.
#pragma once

#include "rk_launch.hpp"
#include "rk_order.hpp"

namespace rkmi {

enum : int32_t { kSysTape = 4 };

// Tape layout for n systems, cap steps, period K, N unknowns, each system's
// records contiguous (a lane reads its own steps in sequence, so one cache
// line serves 16 steps whichever systems the lanes of a wave hold):
//   count int32 [n] | h double [n][hs] | s int32 [n][hs] | y double [n][cs]
//   | the cost order's working area (an order_layout from off_order)
// with hs = cap and cs = (cap/K + 1) N, each rounded up to a multiple of 16;
// system i's checkpoint c is y[i][c N .. c N + N - 1].
struct TapeLayout {
  size_t off_h, off_s, off_ckpt, off_order, bytes;
  int64_t hs, cs;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int64_t kTapeRowAlign = 16;

inline TapeLayout tape_layout(int64_t n, int64_t cap, int32_t K, int N) {
  TapeLayout t;
  t.hs = (cap + kTapeRowAlign - 1) / kTapeRowAlign * kTapeRowAlign;
  t.cs = ((cap / K + 1) * N + kTapeRowAlign - 1) / kTapeRowAlign * kTapeRowAlign;
  t.off_h = align256(sizeof(int32_t) * (size_t)n);
  t.off_s = t.off_h + align256(sizeof(double) * (size_t)t.hs * (size_t)n);
  t.off_ckpt = t.off_s + align256(sizeof(int32_t) * (size_t)t.hs * (size_t)n);
  t.off_order = align256(t.off_ckpt + sizeof(double) * (size_t)t.cs * (size_t)n);
  t.bytes = t.off_order + order_layout(0, n).bytes;
  return t;
}

struct TapeView {
  int32_t* count;   // accepted steps per system, -1 when they exceeded cap
  double* h;        // [n][hs]
  int32_t* s;       // [n][hs]
  double* ckpt;     // [n][cs]
  int64_t n, cap, hs, cs;
  int32_t K;
  RKMI_HD double hstep(int64_t i, int64_t k) const { return h[i * hs + k]; }
  RKMI_HD int32_t sstep(int64_t i, int64_t k) const { return s[i * hs + k]; }
  // checkpoint c of system i (N doubles)
  RKMI_HD double* ck(int64_t i, int64_t c, int N) const { return ckpt + i * cs + c * N; }
};

inline TapeView tape_view(const TapeArgs& a, int64_t n, int N) {
  const TapeLayout L = tape_layout(n, a.cap, a.K, N);
  unsigned char* b = static_cast<unsigned char*>(a.tape);
  return TapeView{reinterpret_cast<int32_t*>(b), reinterpret_cast<double*>(b + L.off_h),
                  reinterpret_cast<int32_t*>(b + L.off_s),
                  reinterpret_cast<double*>(b + L.off_ckpt), n, a.cap, L.hs, L.cs, a.K};
}

// Forward recorder of system i.
template <int N>
struct TapeRec {
  TapeView T;
  int64_t i;
  bool full;
  int32_t phase = 0;     // accepted steps since the last checkpoint (nstep mod K)
  int64_t ck = 0;        // checkpoints written (nstep / K)
  template <class V>
  RKMI_HD void checkpoint(int64_t c, const V& y) {
#pragma unroll
    for (int k = 0; k < N; ++k) T.ck(i, c, N)[k] = y[k];
  }
  template <class V>
  RKMI_HD void accept(double h, int m, const V& yn, int64_t nstep) {
    const int64_t k = nstep - 1;
    if (full || k >= T.cap) {
      full = true;
      return;
    }
    T.h[i * T.hs + k] = h;
    T.s[i * T.hs + k] = m;
    if (++phase == T.K) {          // nstep % K == 0: checkpoint nstep / K
      phase = 0;
      checkpoint(++ck, yn);
    }
  }
};

// Stage records held in LDS (the rest in the lane's workspace columns): the
// reverse sweep writes and reads a step's records once each, and steps of up
// to this many stages (nearly all) keep them on chip.
constexpr int kAdjLdsStages = 2;

// Stage records of one step: record j (1..s) holds w_{j-1} and (mu_j, nu_j,
// mut_j, gt_j); record 1 holds w_0 and mut_1.  Records 1..kAdjLdsStages are
// in the lane's LDS column (lcol), the others in its workspace column (col);
// both with stride kLdsStride.
template <int N>
struct StageRecorder {
  static constexpr bool kStopAtLast = true;
  static constexpr int kRows = N + 4;
  double* lcol;
  double* col;
  RKMI_HD double* rec(int j) const {
    return j <= kAdjLdsStages ? lcol + (int64_t)(j - 1) * kRows * kLdsStride
                              : col + (int64_t)(j - 1) * kRows * kLdsStride;
  }
  template <class V>
  RKMI_HD void first(const V& w0, double mut1) {
    double* const r = rec(1);
#pragma unroll
    for (int k = 0; k < N; ++k) r[k * kLdsStride] = w0[k];
    r[N * kLdsStride] = mut1;
  }
  template <class V>
  RKMI_HD void stage(int j, const V& w, double mu, double nu, double mut, double gt) {
    double* r = rec(j);
#pragma unroll
    for (int k = 0; k < N; ++k) r[k * kLdsStride] = w[k];
    r[N * kLdsStride] = mu;
    r[(N + 1) * kLdsStride] = nu;
    r[(N + 2) * kLdsStride] = mut;
    r[(N + 3) * kLdsStride] = gt;
  }
};

// RKCK stage arguments z_2..z_6 of one step into rows (i - 1) N .. of the
// lane's columns (z_1 = y is stored by the caller).
template <int N>
struct RkckStageRecorder {
  double* col;
  template <class V>
  RKMI_HD void rkck_stage(int i, const V& z) {
    double* r = col + (int64_t)(i - 1) * N * kLdsStride;
#pragma unroll
    for (int k = 0; k < N; ++k) r[k * kLdsStride] = z[k];
  }
};

// Rows of a lane's adjoint columns.  RKC: max_stages stage records, K step
// starts.  RKCK: six stage arguments z_i, their adjoints zbar_i, K step starts.
template <class Prob, int Method>
RKMI_HD int64_t adjoint_rows(int max_stages, int K) {
  if (Method == kMethodRkck) return (int64_t)12 * Prob::N + (int64_t)K * Prob::N;
  return (int64_t)max_stages * (Prob::N + 4) + (int64_t)K * Prob::N;
}

// Forward integration of system i with its tape (RKCK records s = 6).
template <class Prob, int Method>
RKMI_HD void taped_system(const typename Prob::Params& prm, int64_t n, int64_t i,
                          const double* y0, double* y1, const double* g, const Ctl& c,
                          int32_t* status, int32_t* stats, const TapeView& T, double* slot) {
  TapeRec<Prob::N> R{T, i, false};
  Driver<Prob, Method, TapeRec<Prob::N>> D;
  D.rec = &R;
  const bool go = D.start(prm, c, n, i, y0, g, slot);
  R.checkpoint(0, D.state());
  if (go)
    while (D.attempt(prm, c, slot)) {
    }
  D.finish(n, i, y1, status, stats);
  T.count[i] = R.full ? -1 : (int32_t)D.accepted();
}

// Reverse sweep of system i; returns its status.  lambda = w[:, i] on entry,
// dL/dy0 and the per-system dL/dtheta on exit (NaN when the tape is
// incomplete).
template <class Prob>
RKMI_HD int32_t adjoint_system(const typename Prob::Params& prm, int64_t n, int64_t i,
                               const double* g, const TapeView& T, int max_stages,
                               const double* w, double* dy0, double* dth, double* slot,
                               double* col, double* lcol) {
  constexpr int N = Prob::N, NT = Prob::kNTheta;
  using V = RegVec<N>;
  typename Prob::Lane L;
  Prob::init(L, prm, g, i, n, slot);
  const int64_t M = T.count[i];
  V lam;
  double th[NT];
#pragma unroll
  for (int k = 0; k < N; ++k) lam[k] = w[(int64_t)k * n + i];
#pragma unroll
  for (int q = 0; q < NT; ++q) th[q] = 0.0;
  int32_t st = M < 0 ? kSysTape : kSysOk;
  double* const ys = col + (int64_t)max_stages * StageRecorder<N>::kRows * kLdsStride;
  StageRecorder<N> Rec{lcol, col};
  for (int64_t seg = M > 0 ? (M - 1) / T.K : -1; st == kSysOk && seg >= 0; --seg) {
    const int64_t k0 = seg * T.K;
    const int64_t k1 = (k0 + T.K < M) ? k0 + T.K : M;
    // step-start states of the segment, from its checkpoint
    V y;
#pragma unroll
    for (int r = 0; r < N; ++r) y[r] = T.ck(i, seg, N)[r];
    for (int64_t k = k0; k < k1; ++k) {
      double* const yk = ys + (k - k0) * N * kLdsStride;
#pragma unroll
      for (int r = 0; r < N; ++r) yk[r * kLdsStride] = y[r];
      if (k + 1 < k1) {
        V F, yn;
        Prob::rhs(L, prm, y, F);
        rkc_step<Prob>(L, prm, y, F, T.hstep(i, k), T.sstep(i, k), yn, slot);
        y = yn;
      }
    }
    for (int64_t k = k1 - 1; k >= k0; --k) {
      const int sk = T.sstep(i, k);
      const double hk = T.hstep(i, k);
      if (sk < 2 || sk > max_stages) {
        st = kSysTape;
        break;
      }
      const double* const yk = ys + (k - k0) * N * kLdsStride;
#pragma unroll
      for (int r = 0; r < N; ++r) y[r] = yk[r * kLdsStride];
      {
        V F, wlast;
        Prob::rhs(L, prm, y, F);
        rkc_step<Prob, StageRecorder<N>>(L, prm, y, F, hk, sk, wlast, slot, &Rec);
      }
      V cur, m1, m2, A0, f0b, u, jtu, Wv;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        cur[r] = lam[r];
        m1[r] = 0.0;
        m2[r] = 0.0;
        A0[r] = 0.0;
        f0b[r] = 0.0;
      }
      for (int j = sk; j >= 2; --j) {
        const double* const rj = Rec.rec(j);
#pragma unroll
        for (int r = 0; r < N; ++r) Wv[r] = rj[r * kLdsStride];
        const double mu = rj[N * kLdsStride], nu = rj[(N + 1) * kLdsStride];
        const double mut = rj[(N + 2) * kLdsStride], gt = rj[(N + 3) * kLdsStride];
        const double c0 = 1.0 - mu - nu;
        const double gh = gt * hk, mh = mut * hk;
        if (j > 2) {
#pragma unroll
          for (int r = 0; r < N; ++r) {
            A0[r] += c0 * cur[r];
            m1[r] += mu * cur[r];
            m2[r] += nu * cur[r];
            f0b[r] += gh * cur[r];
            u[r] = mh * cur[r];
          }
        } else {
          // w_{j-2} is w_0
#pragma unroll
          for (int r = 0; r < N; ++r) {
            A0[r] += c0 * cur[r];
            m1[r] += mu * cur[r];
            A0[r] += nu * cur[r];
            f0b[r] += gh * cur[r];
            u[r] = mh * cur[r];
          }
        }
        Prob::vjp(L, prm, Wv, u, jtu, th);
#pragma unroll
        for (int r = 0; r < N; ++r) {
          cur[r] = m1[r] + jtu[r];
          m1[r] = m2[r];
          m2[r] = 0.0;
        }
      }
      const double* const r1 = Rec.rec(1);
#pragma unroll
      for (int r = 0; r < N; ++r) Wv[r] = r1[r * kLdsStride];
      const double mh1 = r1[N * kLdsStride] * hk;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        A0[r] += cur[r];
        f0b[r] += mh1 * cur[r];
      }
      Prob::vjp(L, prm, Wv, f0b, jtu, th);
#pragma unroll
      for (int r = 0; r < N; ++r) lam[r] = A0[r] + jtu[r];
    }
  }
  const double nan = crm::from_bits(0x7ff8000000000000ull);
#pragma unroll
  for (int k = 0; k < N; ++k) dy0[(int64_t)k * n + i] = st == kSysOk ? lam[k] : nan;
  if (dth)
#pragma unroll
    for (int q = 0; q < NT; ++q) dth[(int64_t)q * n + i] = st == kSysOk ? th[q] : nan;
  return st;
}

// Reverse sweep of system i under RKCK, as adjoint_system.
template <class Prob>
RKMI_HD int32_t adjoint_system_rkck(const typename Prob::Params& prm, int64_t n, int64_t i,
                                    const double* g, const TapeView& T, const double* w,
                                    double* dy0, double* dth, double* slot, double* col) {
  constexpr int N = Prob::N, NT = Prob::kNTheta;
  using V = RegVec<N>;
  typename Prob::Lane L;
  Prob::init(L, prm, g, i, n, slot);
  const int64_t M = T.count[i];
  V lam;
  double th[NT];
#pragma unroll
  for (int k = 0; k < N; ++k) lam[k] = w[(int64_t)k * n + i];
#pragma unroll
  for (int q = 0; q < NT; ++q) th[q] = 0.0;
  int32_t st = M < 0 ? kSysTape : kSysOk;
  double* const zc = col;                                 // z_1..z_6
  double* const zbc = col + (int64_t)6 * N * kLdsStride;  // zbar_1..zbar_6
  double* const ys = col + (int64_t)12 * N * kLdsStride;  // step starts of a segment
  for (int64_t seg = M > 0 ? (M - 1) / T.K : -1; st == kSysOk && seg >= 0; --seg) {
    const int64_t k0 = seg * T.K;
    const int64_t k1 = (k0 + T.K < M) ? k0 + T.K : M;
    V y;
#pragma unroll
    for (int r = 0; r < N; ++r) y[r] = T.ck(i, seg, N)[r];
    for (int64_t k = k0; k < k1; ++k) {
      double* const yk = ys + (k - k0) * N * kLdsStride;
#pragma unroll
      for (int r = 0; r < N; ++r) yk[r * kLdsStride] = y[r];
      if (k + 1 < k1) {
        V F, yt, ye;
        Prob::rhs(L, prm, y, F);
        rkck_trial<Prob>(L, prm, y, F, T.hstep(i, k), yt, ye, slot);
        y = yt;
      }
    }
    for (int64_t k = k1 - 1; k >= k0; --k) {
      const double hk = T.hstep(i, k);
      const double* const yk = ys + (k - k0) * N * kLdsStride;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        y[r] = yk[r * kLdsStride];
        zc[r * kLdsStride] = y[r];
      }
      {
        V F, yt, ye;
        Prob::rhs(L, prm, y, F);
        RkckStageRecorder<N> R{zc};
        rkck_trial<Prob, RkckStageRecorder<N>>(L, prm, y, F, hk, yt, ye, slot, &R);
      }
      // kbar_i = c_i lambda + sum_{i' > i} b_i'i zbar_i' is formed when stage i
      // is reached (accumulated from i' = 6 down, the order in which the
      // transposed sweep adds the terms), from the zbar_i' kept in the lane's
      // columns
      V yb, u, z, zb;
#pragma unroll
      for (int r = 0; r < N; ++r) yb[r] = lam[r];
      for (int si = 5; si >= 0; --si) {
        const double* const zi = zc + (int64_t)si * N * kLdsStride;
#pragma unroll
        for (int r = 0; r < N; ++r) {
          double kb = ck::kC[si] * lam[r];
          for (int ip = 5; ip > si; --ip) kb += ck::kB[ip][si] * zbc[((int64_t)ip * N + r) * kLdsStride];
          u[r] = hk * kb;
          z[r] = zi[r * kLdsStride];
        }
        Prob::vjp(L, prm, z, u, zb, th);
        double* const zbi = zbc + (int64_t)si * N * kLdsStride;
#pragma unroll
        for (int r = 0; r < N; ++r) {
          yb[r] += zb[r];
          zbi[r * kLdsStride] = zb[r];
        }
      }
      lam = yb;
    }
  }
  const double nan = crm::from_bits(0x7ff8000000000000ull);
#pragma unroll
  for (int k = 0; k < N; ++k) dy0[(int64_t)k * n + i] = st == kSysOk ? lam[k] : nan;
  if (dth)
#pragma unroll
    for (int q = 0; q < NT; ++q) dth[(int64_t)q * n + i] = st == kSysOk ? th[q] : nan;
  return st;
}

template <class Prob, int Method>
__global__ __launch_bounds__(kLdsStride)
__attribute__((amdgpu_waves_per_eu(WavesPerEu<Prob>::value))) void taped_kernel(typename Prob::Params prm, int64_t n,
                                                           const double* y0, double* y1,
                                                           const double* __restrict__ g, Ctl c,
                                                           int32_t* __restrict__ status,
                                                           int32_t* __restrict__ stats,
                                                           TapeView T,
                                                           const int32_t* __restrict__ order) {
  __shared__ double lds[kernel_lds_doubles<Prob, Method>() * kLdsStride];
  const int64_t q = (int64_t)blockIdx.x * kLdsStride + threadIdx.x;
  if (q >= n) return;
  const int64_t i = order ? (int64_t)order[q] : q;   // lane q integrates system order[q]
  taped_system<Prob, Method>(prm, n, i, y0, y1, g, c, status, stats, T, lds + threadIdx.x);
}

// LDS doubles per lane of the reverse kernel: the problem's slot, then (RKC)
// the on-chip stage records.
template <class Prob, int Method>
constexpr int adjoint_lds_doubles() {
  return kernel_lds_doubles<Prob, Method>() +
         (Method == kMethodRkc ? kAdjLdsStages * StageRecorder<Prob::N>::kRows : 0);
}

template <class Prob, int Method>
__global__ __launch_bounds__(kLdsStride) void adjoint_kernel(typename Prob::Params prm, int64_t n,
                                                             const double* __restrict__ g,
                                                             TapeView T, int max_stages,
                                                             const double* __restrict__ w,
                                                             double* __restrict__ dy0,
                                                             double* __restrict__ dth,
                                                             int32_t* __restrict__ status,
                                                             double* cols,
                                                             const int32_t* __restrict__ order) {
  __shared__ double lds[adjoint_lds_doubles<Prob, Method>() * kLdsStride];
  const int64_t q = (int64_t)blockIdx.x * kLdsStride + threadIdx.x;
  if (q >= n) return;
  const int64_t i = order ? (int64_t)order[q] : q;   // lane q sweeps system order[q]
  double* const col = cols +
                      (int64_t)blockIdx.x * adjoint_rows<Prob, Method>(max_stages, T.K) * kLdsStride +
                      threadIdx.x;
  int32_t st;
  if constexpr (Method == kMethodRkck)
    st = adjoint_system_rkck<Prob>(prm, n, i, g, T, w, dy0, dth, lds + threadIdx.x, col);
  else
    st = adjoint_system<Prob>(prm, n, i, g, T, max_stages, w, dy0, dth, lds + threadIdx.x, col,
                              lds + kernel_lds_doubles<Prob, Method>() * kLdsStride + threadIdx.x);
  if (status) status[i] = st;
}

// Bytes of the adjoint's per-lane columns for n systems (one block per 64
// systems); the workspace holds them followed by an order_layout.
template <class Prob, int Method>
int64_t adjoint_column_bytes(int64_t n, int max_stages, int K) {
  const int64_t blocks = (n + kLdsStride - 1) / kLdsStride;
  return blocks * adjoint_rows<Prob, Method>(max_stages, K) * kLdsStride * (int64_t)sizeof(double);
}

// The reverse sweep hands systems to lanes in decreasing order of their
// accepted steps, read from the tape (the sweep's cost is proportional to
// them): the cost order with exact keys and no pilot.
template <int = 0>
__global__ void adjoint_keys_kernel(const int32_t* __restrict__ count, int64_t n,
                                    int32_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  keys[(int64_t)kStAccept * n + i] = count[i] > 0 ? count[i] : 0;
  keys[(int64_t)kStReject * n + i] = 0;
}

template <class Prob>
int launch_taped(const LaunchArgs* a, const TapeArgs* t, void* stream) {
  static_assert(!Prob::kColumns, "the adjoint keeps the system's vectors in registers");
  const int64_t blocks = (a->n + kLdsStride - 1) / kLdsStride;
  if (blocks <= 0) return kLaunchOk;
  if (blocks > 0x7fffffffLL) return kLaunchInvalid;
  if (!t->tape || t->K < 1 || t->cap < 0 ||
      t->tape_bytes < tape_layout(a->n, t->cap, t->K, Prob::N).bytes)
    return kLaunchWorkspace;
  const TapeView T = tape_view(*t, a->n, Prob::N);
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (a->method == kMethodRkck)
    taped_kernel<Prob, kMethodRkck><<<dim3((unsigned)blocks), dim3(kLdsStride), 0, s>>>(
        a->prm, a->n, a->y0, a->y1, a->g, a->ctl, a->status, a->stats, T, a->order);
  else
    taped_kernel<Prob, kMethodRkc><<<dim3((unsigned)blocks), dim3(kLdsStride), 0, s>>>(
        a->prm, a->n, a->y0, a->y1, a->g, a->ctl, a->status, a->stats, T, a->order);
  return hipGetLastError() == hipSuccess ? kLaunchOk : kLaunchHip;
}

template <class Prob>
int launch_adjoint(const AdjointArgs* a, void* stream) {
  const int64_t blocks = (a->n + kLdsStride - 1) / kLdsStride;
  if (blocks <= 0) return kLaunchOk;
  if (blocks > 0x7fffffffLL) return kLaunchInvalid;
  if (!a->tape.tape || a->tape.K < 1 || a->tape.cap < 0 ||
      a->tape.tape_bytes < tape_layout(a->n, a->tape.cap, a->tape.K, Prob::N).bytes)
    return kLaunchInvalid;
  const bool ck = a->method == kMethodRkck;
  const int64_t cols = ck ? adjoint_column_bytes<Prob, kMethodRkck>(a->n, 0, a->tape.K)
                          : adjoint_column_bytes<Prob, kMethodRkc>(a->n, a->max_stages,
                                                                   a->tape.K);
  if (a->n > 0x7fffffffLL) return kLaunchInvalid;
  const OrderLayout L = order_layout((size_t)cols, a->n);
  if ((!ck && a->max_stages < 2) || !a->ws || a->ws_bytes < L.bytes) return kLaunchWorkspace;
  const TapeView T = tape_view(a->tape, a->n, Prob::N);
  const hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* const ws = static_cast<unsigned char*>(a->ws);
  int32_t* const keys = reinterpret_cast<int32_t*>(ws + L.stats);
  int32_t* const order = reinterpret_cast<int32_t*>(ws + L.order);
  int32_t* const hist = reinterpret_cast<int32_t*>(ws + L.hist);
  int32_t* const offs = reinterpret_cast<int32_t*>(ws + L.offs);
  const unsigned chunks = (unsigned)((a->n + kOrderChunk - 1) / kOrderChunk);
  adjoint_keys_kernel<><<<dim3((unsigned)((a->n + 255) / 256)), dim3(256), 0, s>>>(T.count, a->n,
                                                                                   keys);
  order_clear_kernel<><<<1, 256, 0, s>>>(hist);
  order_hist_kernel<><<<chunks, kOrderChunkThreads, 0, s>>>(keys, a->n, hist);
  order_scan_kernel<><<<1, kOrderScanThreads, 0, s>>>(hist, offs);
  order_scatter_kernel<><<<chunks, kOrderChunkThreads, 0, s>>>(keys, a->n, offs, order);
  if (ck)
    adjoint_kernel<Prob, kMethodRkck><<<dim3((unsigned)blocks), dim3(kLdsStride), 0, s>>>(
        a->prm, a->n, a->g, T, 0, a->w, a->dy0, a->dth, a->status, static_cast<double*>(a->ws),
        order);
  else
    adjoint_kernel<Prob, kMethodRkc><<<dim3((unsigned)blocks), dim3(kLdsStride), 0, s>>>(
        a->prm, a->n, a->g, T, a->max_stages, a->w, a->dy0, a->dth, a->status,
        static_cast<double*>(a->ws), order);
  return hipGetLastError() == hipSuccess ? kLaunchOk : kLaunchHip;
}

// Host builds of the same per-system code (test hooks over host arrays).
template <class Prob>
int host_taped(const LaunchArgs* a, const TapeArgs* t) {
  if (!t->tape || t->K < 1 || t->tape_bytes < tape_layout(a->n, t->cap, t->K, Prob::N).bytes)
    return kLaunchWorkspace;
  const TapeView T = tape_view(*t, a->n, Prob::N);
  std::vector<double> slot((size_t)kernel_lds_doubles<Prob, kMethodRkc>() * kLdsStride);
  for (int64_t i = 0; i < a->n; ++i) {
    if (a->method == kMethodRkck)
      taped_system<Prob, kMethodRkck>(a->prm, a->n, i, a->y0, a->y1, a->g, a->ctl, a->status,
                                      a->stats, T, slot.data());
    else
      taped_system<Prob, kMethodRkc>(a->prm, a->n, i, a->y0, a->y1, a->g, a->ctl, a->status,
                                     a->stats, T, slot.data());
  }
  return kLaunchOk;
}

template <class Prob>
int host_adjoint(const AdjointArgs* a) {
  const bool ck = a->method == kMethodRkck;
  if (!a->tape.tape || a->tape.K < 1 || (!ck && a->max_stages < 2) ||
      a->tape.tape_bytes < tape_layout(a->n, a->tape.cap, a->tape.K, Prob::N).bytes)
    return kLaunchInvalid;
  const TapeView T = tape_view(a->tape, a->n, Prob::N);
  std::vector<double> slot((size_t)kernel_lds_doubles<Prob, kMethodRkc>() * kLdsStride);
  const int64_t rows = ck ? adjoint_rows<Prob, kMethodRkck>(0, a->tape.K)
                          : adjoint_rows<Prob, kMethodRkc>(a->max_stages, a->tape.K);
  std::vector<double> col((size_t)rows * kLdsStride);
  std::vector<double> lcol((size_t)kAdjLdsStages * StageRecorder<Prob::N>::kRows * kLdsStride);
  for (int64_t i = 0; i < a->n; ++i) {
    const int32_t st =
        ck ? adjoint_system_rkck<Prob>(a->prm, a->n, i, a->g, T, a->w, a->dy0, a->dth,
                                       slot.data(), col.data())
           : adjoint_system<Prob>(a->prm, a->n, i, a->g, T, a->max_stages, a->w, a->dy0,
                                  a->dth, slot.data(), col.data(), lcol.data());
    if (a->status) a->status[i] = st;
  }
  return kLaunchOk;
}

}  // namespace rkmi
