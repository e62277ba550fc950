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
// driver, so they live in the lane's workspace columns (the column tier).
#include "rk_launch.hpp"

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

}  // namespace rkmi

extern "C" int rkmi_pleiades_launch(const rkmi::LaunchArgs* a, void* s) {
  return rkmi::launch<rkmi::PleiadesProblem>(a, s);
}

extern "C" int rkmi_pleiades_host(const rkmi::LaunchArgs* a) {
  return rkmi::host_run<rkmi::PleiadesProblem>(a);
}

extern "C" int64_t rkmi_pleiades_workspace(int method, int schedule, int64_t n) {
  return rkmi::workspace<rkmi::PleiadesProblem>(method, schedule, n);
}
