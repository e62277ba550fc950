// rk_pleiades.hip -- the Pleiades problem (Sec. 4.1): seven bodies of mass
// m_i = i moving in the plane under their mutual gravitation, as 28
// first-order equations (z, w)' = (w, f(z)) with z = (x_1..x_7, y_1..y_7):
//   x_i'' = sum_{j != i} m_j (x_j - x_i) / r_ij,   y_i'' likewise,
//   r_ij = ((x_i - x_j)^2 + (y_i - y_j)^2)^(3/2)   (the y difference squared);
// no per-system parameters.  r_ij^(3/2) is formed as d2 sqrt(d2) and the
// division by it as a multiplication by its reciprocal, once per pair (the
// pair's value is the same bits for (i, j) and (j, i): the squared differences
// of negated operands are equal).  Each body's sums run over j in increasing
// order from zero.  Its 28-vectors are too many for registers in the RKCK
// driver: one lane per system keeps them in workspace columns (the column
// tier, plain and persistent schedules), and the group variant spreads a
// system over eight lanes (the group schedule, the default).
#include "rk_launch.hpp"
#include "rk_group.hpp"

namespace rkmi {

struct PleiadesProblem {
  static constexpr int N = 28;
  static constexpr bool kColumns = true;
  static constexpr int kGroupLanes = 1;
  static constexpr int kLaneDoubles = 0;
  using Params = const double*;
  struct Lane {};
  RKMI_HD static void init(Lane&, const Params&, const double* __restrict__, int64_t, int64_t,
                           double*) {}
  template <class VI, class VO>
  RKMI_HD static void rhs(const Lane&, const Params&, const VI& y, VO& f) {
    double x[7], yy[7], rinv[7][7];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      x[i] = y[i];
      yy[i] = y[7 + i];
    }
#pragma unroll
    for (int i = 0; i < 14; ++i) f[i] = y[14 + i];
#pragma unroll
    for (int i = 0; i < 7; ++i)
#pragma unroll
      for (int j = i + 1; j < 7; ++j) {
        const double d2 = (x[i] - x[j]) * (x[i] - x[j]) + (yy[i] - yy[j]) * (yy[i] - yy[j]);
        rinv[i][j] = 1.0 / (d2 * sqrt(d2));
        rinv[j][i] = rinv[i][j];
      }
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      double ax = 0.0, ay = 0.0;
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        if (j == i) continue;
        const double mj = (double)(j + 1);
        ax += (mj * (x[j] - x[i])) * rinv[i][j];
        ay += (mj * (yy[j] - yy[i])) * rinv[i][j];
      }
      f[14 + i] = ax;
      f[21 + i] = ay;
    }
  }
};

// Group variant: lane r < 7 of a group of eight holds body r's unknowns
// (x_r, y_r, x_r', y_r') in registers; lane 7 holds none.  An evaluation
// writes the positions to the group's LDS area; the 21 pair values
// 1 / (d2 sqrt(d2)) are formed once each, three per lane (pair p by lane p mod
// 7, with the smaller body index first as the one-lane code forms them), and
// stored for both orders; each body's lane then sums its terms in the one-lane
// order, so results equal the one-lane kernels.
struct PleiadesPairs {
  int i[21], j[21];
  constexpr PleiadesPairs() : i(), j() {
    int p = 0;
    for (int a = 0; a < 7; ++a)
      for (int b = a + 1; b < 7; ++b) {
        i[p] = a;
        j[p] = b;
        ++p;
      }
  }
};
inline constexpr PleiadesPairs kPleiadesPairs{};

struct PleiadesGroup {
  static constexpr int N = 28;
  static constexpr int NR = 0;
  static constexpr int kL = 8;
  static constexpr int kGroupLanes = 8;
  static constexpr bool kColumns = false;
  static constexpr int kLaneDoubles = 0;
  static constexpr int S = 4;
  static constexpr bool kOwnRhs = true;
  static constexpr int kOffPos = 0;               // x_1..x_7, y_1..y_7
  static constexpr int kOffPair = 14;             // 1 / r_ij at i * 7 + j
  static constexpr int kOffRed = kOffPair + 50;   // norm scratch, N doubles (16-byte aligned)
  static constexpr int kLdsPerSystem = kOffRed + N;
  static constexpr int kSp[S * kL] = {0,  1,  2,  3,  4,  5,  6,  -1,     // x_r
                                      7,  8,  9,  10, 11, 12, 13, -1,     // y_r
                                      14, 15, 16, 17, 18, 19, 20, -1,     // x_r'
                                      21, 22, 23, 24, 25, 26, 27, -1};    // y_r'
  using Params = const double*;
  struct Lane {};
  __device__ static void init(Lane&, const Params&, const double* __restrict__, int64_t, int64_t,
                              const Grp<PleiadesGroup>&) {}
  __device__ static void rhs(const Lane&, const Grp<PleiadesGroup>& x, const double (&y)[S],
                             double (&f)[S]) {
    double* const P = x.lds + kOffPos;
    double* const R = x.lds + kOffPair;
    const bool body = x.r < 7;
    if (body) {
      P[x.r] = y[0];
      P[7 + x.r] = y[1];
    }
    group_sync();
    if (body) {
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int p = x.r + 7 * t;
        const int a = kPleiadesPairs.i[p], b = kPleiadesPairs.j[p];
        const double xa = P[a], xb = P[b], ya = P[7 + a], yb = P[7 + b];
        const double d2 = (xa - xb) * (xa - xb) + (ya - yb) * (ya - yb);
        const double rinv = 1.0 / (d2 * sqrt(d2));
        R[a * 7 + b] = rinv;
        R[b * 7 + a] = rinv;
      }
    }
    group_sync();
    double ax = 0.0, ay = 0.0;
    if (body) {
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        if (j == x.r) continue;
        const double rinv = R[x.r * 7 + j];
        const double mj = (double)(j + 1);
        ax += (mj * (P[j] - y[0])) * rinv;
        ay += (mj * (P[7 + j] - y[1])) * rinv;
      }
    }
    f[0] = body ? y[2] : 0.0;
    f[1] = body ? y[3] : 0.0;
    f[2] = ax;
    f[3] = ay;
    group_sync();
  }
};

}  // namespace rkmi

extern "C" int rkmi_pleiades_launch(const rkmi::LaunchArgs* a, void* s) {
  return rkmi::launch_with_group<rkmi::PleiadesProblem, rkmi::PleiadesGroup>(a, s);
}

extern "C" int rkmi_pleiades_host(const rkmi::LaunchArgs* a) {
  return rkmi::host_run<rkmi::PleiadesProblem>(a);
}

extern "C" int64_t rkmi_pleiades_workspace(int method, int schedule, int64_t n) {
  return rkmi::workspace_with_group<rkmi::PleiadesProblem, rkmi::PleiadesGroup>(method, schedule,
                                                                                n);
}
