// rk_abi.hip -- the C ABI declared in include/rkmi.h: argument checks, problem
// handles and dispatch to the compiled kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rkmi.h"
#include "rk_launch.hpp"

extern "C" int rkmi_vdp_launch(const rkmi::LaunchArgs* a, void* s);
extern "C" int rkmi_vdp_host(const rkmi::LaunchArgs* a);
extern "C" int64_t rkmi_vdp_workspace(int method, int schedule, int64_t n);

namespace rkmi {
extern const GenEntry kGenRegistry[];
extern const int kGenRegistrySize;
}  // namespace rkmi

namespace {

constexpr int kMaxDevices = 64;
constexpr int64_t kDefaultMaxSteps = 10000000;

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

enum Kind { kVdp = 1, kMassAction = 3 };

}  // namespace

struct rk_problem_s {
  int kind = 0;
  int n_eq = 0, n_param = 0, n_theta = 0, n_rx = 0;
  rkmi::launch_fn launch = nullptr;
  rkmi::host_fn host = nullptr;
  rkmi::workspace_fn workspace = nullptr;
  std::vector<double> host_prm;        // uniform problem data, device layout
  double* dev_prm[kMaxDevices] = {};   // per-device copies, made on first use
  std::mutex mu;
};

namespace {

// Device copy of the problem's uniform data on the current device.
int problem_device_data(rk_problem p, const double** out) {
  *out = nullptr;
  if (p->host_prm.empty()) return RK_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(RK_EHIP, "no usable current HIP device");
  std::lock_guard<std::mutex> lock(p->mu);
  if (!p->dev_prm[dev]) {
    void* d = nullptr;
    const size_t bytes = p->host_prm.size() * sizeof(double);
    if (hipMalloc(&d, bytes) != hipSuccess) return fail(RK_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    if (hipMemcpy(d, p->host_prm.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d);
      return fail(RK_EHIP, "copy of problem data to the device failed");
    }
    p->dev_prm[dev] = static_cast<double*>(d);
  }
  *out = p->dev_prm[dev];
  return RK_OK;
}

__global__ void empty_interval_kernel(int64_t n, int n_eq, const double* y0,
                                      double* y1, int32_t* __restrict__ status,
                                      int32_t* __restrict__ stats) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (y1 != y0)
    for (int k = 0; k < n_eq; ++k) y1[(int64_t)k * n + i] = y0[(int64_t)k * n + i];
  if (status) status[i] = RK_SYS_OK;
  if (stats)
    for (int r = 0; r < RK_NSTATS; ++r) stats[(int64_t)r * n + i] = 0;
}

// The pointer must be device (or managed) memory of the current device.
int check_device_ptr(const void* ptr, size_t align, const char* name, bool allow_null) {
  if (!ptr) return allow_null ? RK_OK : fail(RK_EINVAL, "%s is NULL", name);
  if (reinterpret_cast<uintptr_t>(ptr) % align)
    return fail(RK_EINVAL, "%s is not %zu-byte aligned", name, align);
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return fail(RK_EINVAL, "%s is not a HIP allocation", name);
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(RK_EINVAL, "%s is not device memory", name);
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (attr.type == hipMemoryTypeDevice && attr.device != dev)
    return fail(RK_EINVAL, "%s lives on device %d, current device is %d", name, attr.device, dev);
  return RK_OK;
}

// Launch arguments and the launch-uniform controls of the drivers.
void fill_args(rkmi::LaunchArgs& a, int method, int64_t n, const double* y0, double* y1,
               const double* g, double t0, double t1, double rtol, double atol, int32_t* status,
               int32_t* stats, void* ws, size_t ws_bytes, const rk_options* opt) {
  a.method = method;
  a.schedule = opt ? opt->schedule : 0;
  a.n = n;
  a.y0 = y0;
  a.y1 = y1;
  a.g = g;
  a.prm = nullptr;
  rkmi::Ctl& c = a.ctl;
  c.t0 = t0;
  c.t1 = t1;
  c.rtol = rtol;
  c.atol = atol;
  c.hmax = std::fabs(t1 - t0);
  c.hmin_rkc = 10.0 * rkmi::kUround * std::fmax(std::fabs(t0), c.hmax);
  c.delta = (atol > 0.0) ? atol / rtol : 1.0e-30;
  c.max_steps = (opt && opt->max_steps > 0) ? opt->max_steps : kDefaultMaxSteps;
  const int mmax = (int)std::round(std::sqrt(rtol / (10.0 * rkmi::kUround)));
  c.mmax = mmax < 2 ? 2 : mmax;
  c.sr_period = (opt && opt->sr_period > 0) ? opt->sr_period : 25;
  c.sr_itmax = (opt && opt->sr_itmax > 0) ? opt->sr_itmax : 50;
  c.refill = (opt && opt->refill > 0) ? (opt->refill > rkmi::kLdsStride ? rkmi::kLdsStride
                                                                        : opt->refill)
                                      : rkmi::kDefaultRefill;
  a.status = status;
  a.stats = stats;
  a.ws = ws;
  a.ws_bytes = ws_bytes;
}

int integrate(int method, rk_problem p, int64_t n, const double* y0, double* y1, const double* g,
              double t0, double t1, double rtol, double atol, int32_t* status, int32_t* stats,
              void* ws, size_t ws_bytes, const rk_options* opt, void* stream) {
  g_err.clear();
  if (!p) return fail(RK_EINVAL, "problem handle is NULL");
  if (n < 0) return fail(RK_EINVAL, "n_sys = %lld is negative", (long long)n);
  if (!std::isfinite(t0) || !std::isfinite(t1) || !(t1 >= t0))
    return fail(RK_EINVAL, "need finite t0 <= t1 (got %g, %g)", t0, t1);
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(RK_EINVAL, "rtol must be positive");
  if (!(atol >= 0.0) || !std::isfinite(atol)) return fail(RK_EINVAL, "atol must be >= 0");
  if (opt) {
    for (int k = 0; k < 6; ++k)
      if (opt->reserved[k]) return fail(RK_EINVAL, "rk_options.reserved must be zero");
    if (opt->schedule < rkmi::kSchedAuto || opt->schedule > rkmi::kSchedPersistent)
      return fail(RK_EUNSUPPORTED, "schedule %d is not available", opt->schedule);
  }
  if (n == 0) return RK_OK;
  int rc;
  if ((rc = check_device_ptr(y0, 8, "y0", false))) return rc;
  if ((rc = check_device_ptr(y1, 8, "y1", false))) return rc;
  if ((rc = check_device_ptr(g, 8, "g", p->n_param == 0))) return rc;
  if ((rc = check_device_ptr(status, 4, "status", true))) return rc;
  if ((rc = check_device_ptr(stats, 4, "stats", true))) return rc;
  if ((rc = check_device_ptr(ws, 8, "ws", true))) return rc;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (t1 == t0) {
    // nothing to integrate: copy the state, zero status and statistics (a
    // kernel rather than memset/memcpy nodes, so the call is graph-capturable)
    const int64_t blocks = (n + 255) / 256;
    empty_interval_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(n, p->n_eq, y0, y1,
                                                                       status, stats);
    if (hipGetLastError() != hipSuccess) return fail(RK_EHIP, "kernel launch failed");
    return RK_OK;
  }
  rkmi::LaunchArgs a;
  fill_args(a, method, n, y0, y1, g, t0, t1, rtol, atol, status, stats, ws, ws_bytes, opt);
  if ((rc = problem_device_data(p, &a.prm))) return rc;
  rc = p->launch(&a, stream);
  if (rc == rkmi::kLaunchWorkspace)
    return fail(RK_EWORKSPACE, "workspace of %zu bytes is too small (rk_workspace_bytes gives "
                "the size this call needs)", ws ? ws_bytes : (size_t)0);
  if (rc == rkmi::kLaunchInvalid) return fail(RK_EINVAL, "too many systems for one launch");
  if (rc) return fail(RK_EHIP, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
  return RK_OK;
}

}  // namespace

extern "C" {

int rk_version(void) { return 100; }

const char* rk_last_error(void) { return g_err.c_str(); }

int rk_problem_create_vdp(rk_problem* out) {
  g_err.clear();
  if (!out) return fail(RK_EINVAL, "out is NULL");
  *out = nullptr;
  rk_problem p = new (std::nothrow) rk_problem_s();
  if (!p) return fail(RK_ENOMEM, "out of host memory");
  p->kind = kVdp;
  p->n_eq = 2;
  p->n_param = 1;
  p->n_theta = 1;
  p->launch = rkmi_vdp_launch;
  p->host = rkmi_vdp_host;
  p->workspace = rkmi_vdp_workspace;
  *out = p;
  return RK_OK;
}

int rk_problem_create_mass_action(const rk_mech_desc* d, rk_problem* out) {
  g_err.clear();
  if (!out) return fail(RK_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d) return fail(RK_EINVAL, "desc is NULL");
  if (d->n_sp <= 0 || d->n_rx <= 0) return fail(RK_EINVAL, "need n_sp > 0 and n_rx > 0");
  if (!d->reac || !d->prod || !d->lnA || !d->beta || !d->Ea || !d->Keq || !d->W)
    return fail(RK_EINVAL, "desc has a NULL array");
  for (int j = 0; j < 2 * d->n_rx; ++j) {
    const bool slot2 = (j & 1);
    for (const int32_t* arr : {d->reac, d->prod}) {
      const int32_t k = arr[j];
      if (k >= d->n_sp || k < (slot2 ? -1 : 0))
        return fail(RK_EINVAL, "species index %d out of range in reaction %d", k, j / 2);
    }
  }
  for (int j = 0; j < d->n_rx; ++j)
    if (!(d->Keq[j] > 0.0) || !std::isfinite(d->lnA[j]) || !std::isfinite(d->beta[j]) ||
        !std::isfinite(d->Ea[j]))
      return fail(RK_EINVAL, "reaction %d has invalid rate parameters", j);
  for (int k = 0; k < d->n_sp; ++k)
    if (!(d->W[k] > 0.0) || !std::isfinite(d->W[k]))
      return fail(RK_EINVAL, "species %d has invalid molar mass", k);
  const rkmi::GenEntry* hit = nullptr;
  for (int e = 0; e < rkmi::kGenRegistrySize; ++e) {
    const rkmi::GenEntry& E = rkmi::kGenRegistry[e];
    if (E.n_sp == d->n_sp && E.n_rx == d->n_rx &&
        !std::memcmp(E.reac, d->reac, sizeof(int32_t) * 2 * d->n_rx) &&
        !std::memcmp(E.prod, d->prod, sizeof(int32_t) * 2 * d->n_rx)) {
      hit = &E;
      break;
    }
  }
  if (!hit)
    return fail(RK_EUNSUPPORTED,
                "no compiled right-hand side for this %d-species / %d-reaction topology; "
                "generate it with the package code generator and rebuild",
                d->n_sp, d->n_rx);
  rk_problem p = new (std::nothrow) rk_problem_s();
  if (!p) return fail(RK_ENOMEM, "out of host memory");
  p->kind = kMassAction;
  p->n_eq = d->n_sp;
  p->n_param = 2;
  p->n_theta = d->n_rx;
  p->n_rx = d->n_rx;
  p->launch = hit->launch;
  p->host = hit->host;
  p->workspace = hit->workspace;
  const int nr = d->n_rx, ns = d->n_sp;
  p->host_prm.resize(4 * nr + 2 * ns);
  for (int j = 0; j < nr; ++j) {
    p->host_prm[j] = d->lnA[j];
    p->host_prm[nr + j] = d->beta[j];
    p->host_prm[2 * nr + j] = d->Ea[j];
    p->host_prm[3 * nr + j] = 1.0 / d->Keq[j];
  }
  for (int k = 0; k < ns; ++k) {
    p->host_prm[4 * nr + k] = d->W[k];
    p->host_prm[4 * nr + ns + k] = 1.0 / d->W[k];
  }
  *out = p;
  return RK_OK;
}

void rk_problem_destroy(rk_problem p) {
  if (!p) return;
  for (int d = 0; d < kMaxDevices; ++d) {
    if (p->dev_prm[d]) {
      int cur = 0;
      (void)hipGetDevice(&cur);
      (void)hipSetDevice(d);
      (void)hipFree(p->dev_prm[d]);
      (void)hipSetDevice(cur);
    }
  }
  delete p;
}

int rk_problem_dims(rk_problem p, int32_t* n_eq, int32_t* n_param, int32_t* n_theta) {
  g_err.clear();
  if (!p) return fail(RK_EINVAL, "problem handle is NULL");
  if (n_eq) *n_eq = p->n_eq;
  if (n_param) *n_param = p->n_param;
  if (n_theta) *n_theta = p->n_theta;
  return RK_OK;
}

size_t rk_workspace_bytes(rk_problem p, int32_t method, int64_t n_sys, const rk_options* opt) {
  g_err.clear();
  if (!p || n_sys <= 0 || (method != RK_METHOD_RKCK && method != RK_METHOD_RKC)) return 0;
  const int schedule = opt ? opt->schedule : rkmi::kSchedAuto;
  if (schedule < rkmi::kSchedAuto || schedule > rkmi::kSchedPersistent) return 0;
  const int64_t b = p->workspace(method == RK_METHOD_RKCK ? rkmi::kMethodRkck : rkmi::kMethodRkc,
                                 schedule, n_sys);
  if (b < 0) {
    fail(RK_EHIP, "could not query the current device");
    return 0;
  }
  return (size_t)b;
}

int rk_integrate_rkck(rk_problem p, int64_t n_sys, const double* y0, double* y1, const double* g,
                      double t0, double t1, double rtol, double atol, int32_t* status,
                      int32_t* stats, void* ws, size_t ws_bytes, const rk_options* opt,
                      void* stream) {
  return integrate(rkmi::kMethodRkck, p, n_sys, y0, y1, g, t0, t1, rtol, atol, status, stats, ws,
                   ws_bytes, opt, stream);
}

int rk_integrate_rkc(rk_problem p, int64_t n_sys, const double* y0, double* y1, const double* g,
                     double t0, double t1, double rtol, double atol, int32_t* status,
                     int32_t* stats, void* ws, size_t ws_bytes, const rk_options* opt,
                     void* stream) {
  return integrate(rkmi::kMethodRkc, p, n_sys, y0, y1, g, t0, t1, rtol, atol, status, stats, ws,
                   ws_bytes, opt, stream);
}

// Test hook, not part of the public ABI: runs the kernels' per-system code on
// the host over HOST arrays, so the CPU test suite can compare the kernels'
// arithmetic with the reference bit for bit.  Integration calls never use it.
int rkmi_test_host_integrate(int32_t method, rk_problem p, int64_t n, const double* y0,
                             double* y1, const double* g, double t0, double t1, double rtol,
                             double atol, int32_t* status, int32_t* stats, int64_t max_steps) {
  g_err.clear();
  if (!p || !p->host || n < 0 || !y0 || !y1 || (p->n_param && !g) || !(t1 > t0) ||
      !(rtol > 0.0) || !(atol >= 0.0))
    return fail(RK_EINVAL, "invalid arguments");
  rk_options o{};
  o.max_steps = max_steps;
  rkmi::LaunchArgs a;
  fill_args(a, method, n, y0, y1, g, t0, t1, rtol, atol, status, stats, nullptr, 0, &o);
  a.prm = p->host_prm.empty() ? nullptr : p->host_prm.data();
  return p->host(&a);
}

}  // extern "C"
