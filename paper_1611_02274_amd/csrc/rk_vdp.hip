// rk_vdp.hip -- van der Pol oscillators, y1' = y2, y2' = mu (1 - y1^2) y2 - y1,
// one parameter g = (mu) per system: the nonstiff RKCK workload.
#include "rk_adjoint.hpp"

namespace rkmi {

struct VdpProblem {
  static constexpr int N = 2;
  static constexpr bool kColumns = false;
  static constexpr int kGroupLanes = 1;
  static constexpr int kLaneDoubles = 0;
  using Params = const double*;
  struct Lane {
    double mu;
  };
  RKMI_HD static void init(Lane& L, const Params&, const double* __restrict__ g, int64_t i,
                           int64_t, double*) {
    L.mu = g[i];
  }
  template <class VI, class VO>
  RKMI_HD static void rhs(const Lane& L, const Params&, const VI& y, VO& f) {
    f[0] = y[1];
    f[1] = L.mu * (1.0 - y[0] * y[0]) * y[1] - y[0];
  }
  // Gershgorin bound of J = [[0, 1], [-2 mu y0 y1 - 1, mu (1 - y0^2)]]: rows
  // summed from zero, the maximum by fmax from zero
  static constexpr bool kGershgorin = true;
  template <class VI>
  RKMI_HD static double gershgorin(const Lane& L, const Params&, const VI& y) {
    const double r0 = (0.0 + fabs(0.0)) + fabs(1.0);
    const double j10 = -2.0 * L.mu * y[0] * y[1] - 1.0;
    const double j11 = L.mu * (1.0 - y[0] * y[0]);
    const double r1 = (0.0 + fabs(j10)) + fabs(j11);
    return fmax(fmax(0.0, r0), r1);
  }
  // vector-Jacobian products, theta = mu: jtu = J(y)^T u, th += (df/dmu)^T u
  static constexpr int kNTheta = 1;
  template <class VI, class VU, class VO>
  RKMI_HD static void vjp(const Lane& L, const Params&, const VI& y, const VU& u, VO& jtu,
                          double (&th)[1]) {
    jtu[0] = u[1] * (-2.0 * L.mu * y[0] * y[1] - 1.0);
    jtu[1] = u[0] + u[1] * L.mu * (1.0 - y[0] * y[0]);
    th[0] += u[1] * (1.0 - y[0] * y[0]) * y[1];
  }
};

}  // namespace rkmi

extern "C" int rkmi_vdp_launch(const rkmi::LaunchArgs* a, void* s) {
  return rkmi::launch<rkmi::VdpProblem>(a, s);
}

extern "C" int rkmi_vdp_host(const rkmi::LaunchArgs* a) {
  return rkmi::host_run<rkmi::VdpProblem>(a);
}

extern "C" int64_t rkmi_vdp_workspace(int method, int schedule, int64_t n) {
  return rkmi::workspace<rkmi::VdpProblem>(method, schedule, n);
}

extern "C" int rkmi_vdp_taped(const rkmi::LaunchArgs* a, const rkmi::TapeArgs* t, void* s) {
  return rkmi::launch_taped<rkmi::VdpProblem>(a, t, s);
}

extern "C" int rkmi_vdp_taped_host(const rkmi::LaunchArgs* a, const rkmi::TapeArgs* t) {
  return rkmi::host_taped<rkmi::VdpProblem>(a, t);
}

extern "C" int rkmi_vdp_adjoint(const rkmi::AdjointArgs* a, void* s) {
  return rkmi::launch_adjoint<rkmi::VdpProblem>(a, s);
}

extern "C" int rkmi_vdp_adjoint_host(const rkmi::AdjointArgs* a) {
  return rkmi::host_adjoint<rkmi::VdpProblem>(a);
}
