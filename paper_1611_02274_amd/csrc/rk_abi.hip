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
#include <utility>
#include <vector>

#include "../../include/rkmi.h"
#include "rk_adjoint.hpp"
#include "rk_batch.hpp"
#include "rk_order.hpp"

extern "C" int rkmi_vdp_launch(const rkmi::LaunchArgs* a, void* s);
extern "C" int rkmi_vdp_host(const rkmi::LaunchArgs* a);
extern "C" int64_t rkmi_vdp_workspace(int method, int schedule, int64_t n);
extern "C" int rkmi_vdp_taped(const rkmi::LaunchArgs* a, const rkmi::TapeArgs* t, void* s);
extern "C" int rkmi_vdp_taped_host(const rkmi::LaunchArgs* a, const rkmi::TapeArgs* t);
extern "C" int rkmi_vdp_adjoint(const rkmi::AdjointArgs* a, void* s);
extern "C" int rkmi_vdp_adjoint_host(const rkmi::AdjointArgs* a);
extern "C" int rkmi_pleiades_launch(const rkmi::LaunchArgs* a, void* s);
extern "C" int rkmi_pleiades_host(const rkmi::LaunchArgs* a);
extern "C" int64_t rkmi_pleiades_workspace(int method, int schedule, int64_t n);

namespace rkmi {
extern const GenEntry kGenRegistry[];
extern const int kGenRegistrySize;
extern const BatchEntry kBatchRegistry[];
extern const int kBatchRegistrySize;
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

enum Kind { kVdp = 1, kMassAction = 3, kPleiades = 4, kMassActionThermal = 5 };

}  // namespace

struct rk_problem_s {
  int kind = 0;
  int n_eq = 0, n_param = 0, n_theta = 0, n_rx = 0;
  rkmi::launch_fn launch = nullptr;
  rkmi::host_fn host = nullptr;
  rkmi::workspace_fn workspace = nullptr;
  rkmi::taped_fn taped = nullptr;
  rkmi::taped_host_fn taped_host = nullptr;
  rkmi::adjoint_fn adjoint = nullptr;
  rkmi::adjoint_host_fn adjoint_host = nullptr;
  int gen_index = -1;                  // row of the network registry
  bool gershgorin = false;             // has the analytic Jacobian (sr_method 1)
  std::vector<double> host_prm;        // uniform problem data, device layout
  double* dev_prm[kMaxDevices] = {};   // per-device copies, made on first use
  std::mutex mu;
};

namespace {

// Device copy of the problem's uniform data on the current device, made on
// first use unless may_alloc is false (then its absence is an error).
int problem_device_data(rk_problem p, const double** out, bool may_alloc = true) {
  *out = nullptr;
  if (p->host_prm.empty()) return RK_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(RK_EHIP, "no usable current HIP device");
  std::lock_guard<std::mutex> lock(p->mu);
  if (!p->dev_prm[dev] && !may_alloc)
    return fail(RK_EINVAL, "the problem's constants are not on device %d yet (the first "
                "allocating call with this problem on the device copies them there)", dev);
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

// The launch-uniform controls of the drivers for [t0, t1].
void fill_ctl(rkmi::Ctl& c, double t0, double t1, double rtol, double atol,
              const rk_options* opt) {
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
  c.sr_method = opt ? opt->sr_method : rkmi::kSrPower;
  c.refill = (opt && opt->refill > 0) ? (opt->refill > rkmi::kLdsStride ? rkmi::kLdsStride
                                                                        : opt->refill)
                                      : rkmi::kDefaultRefill;
  c.align = opt ? (opt->group_align > 64 ? 64 : opt->group_align) : 0;
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
  fill_ctl(a.ctl, t0, t1, rtol, atol, opt);
  a.status = status;
  a.stats = stats;
  a.ws = ws;
  a.ws_bytes = ws_bytes;
  a.order = nullptr;
  a.pilot = 0;
  a.carry = nullptr;
}

int integrate(int method, rk_problem p, int64_t n, const double* y0, double* y1, const double* g,
              double t0, double t1, double rtol, double atol, int32_t* status, int32_t* stats,
              void* ws, size_t ws_bytes, const rk_options* opt, void* stream,
              const rkmi::TapeArgs* tape = nullptr, double* carry = nullptr,
              bool want_carry = false, bool static_ws = false) {
  g_err.clear();
  if (!p) return fail(RK_EINVAL, "problem handle is NULL");
  if (tape && !p->taped)
    return fail(RK_EUNSUPPORTED, "the adjoint is not compiled for this problem (systems of "
                "more than 16 unknowns keep their vectors in workspace columns)");
  if (tape && (tape->K < 1 || tape->cap < 0))
    return fail(RK_EINVAL, "need ckpt_every >= 1 and max_accepted >= 0");
  if (n < 0) return fail(RK_EINVAL, "n_sys = %lld is negative", (long long)n);
  if (!std::isfinite(t0) || !std::isfinite(t1) || !(t1 >= t0))
    return fail(RK_EINVAL, "need finite t0 <= t1 (got %g, %g)", t0, t1);
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(RK_EINVAL, "rtol must be positive");
  if (!(atol >= 0.0) || !std::isfinite(atol)) return fail(RK_EINVAL, "atol must be >= 0");
  if (opt) {
    for (size_t k = 0; k < sizeof(opt->reserved) / sizeof(opt->reserved[0]); ++k)
      if (opt->reserved[k]) return fail(RK_EINVAL, "rk_options.reserved must be zero");
    if (opt->schedule < rkmi::kSchedAuto || opt->schedule > rkmi::kSchedGroup)
      return fail(RK_EUNSUPPORTED, "schedule %d is not available", opt->schedule);
    if (opt->sr_method != rkmi::kSrPower && opt->sr_method != rkmi::kSrGershgorin)
      return fail(RK_EINVAL, "sr_method must be 0 (power method) or 1 (Gershgorin)");
    if (opt->sr_method == rkmi::kSrGershgorin && method == rkmi::kMethodRkc &&
        (!p->gershgorin || tape))
      return fail(RK_EUNSUPPORTED, "the Gershgorin bound needs the analytic Jacobian (van der "
                  "Pol, isothermal networks of up to 16 species) and no tape");
  }
  if (n == 0) return RK_OK;
  int rc;
  if ((rc = check_device_ptr(y0, 8, "y0", false))) return rc;
  if ((rc = check_device_ptr(y1, 8, "y1", false))) return rc;
  if ((rc = check_device_ptr(g, 8, "g", p->n_param == 0))) return rc;
  if ((rc = check_device_ptr(status, 4, "status", true))) return rc;
  if ((rc = check_device_ptr(stats, 4, "stats", true))) return rc;
  if (!static_ws && (rc = check_device_ptr(ws, 8, "ws", true))) return rc;
  if (want_carry && (rc = check_device_ptr(carry, 8, "carry", false))) return rc;
  if (tape) {
    if ((rc = check_device_ptr(tape->tape, 256, "tape", false))) return rc;
    const size_t need = rkmi::tape_layout(n, tape->cap, tape->K, p->n_eq).bytes;
    if (tape->tape_bytes < need)
      return fail(RK_EWORKSPACE, "tape of %zu bytes is too small (%zu needed)", tape->tape_bytes,
                  need);
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (t1 == t0 && !tape && !carry) {
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
  a.carry = carry;
  if ((rc = problem_device_data(p, &a.prm, !static_ws))) return rc;
  if (opt && opt->cost_order && tape) {
    // the pilot (one-lane plain kernel) and the sort work in the tape's own
    // order area; the taped kernel then takes the order map
    const rkmi::TapeLayout tl = rkmi::tape_layout(n, tape->cap, tape->K, p->n_eq);
    rkmi::LaunchArgs t = a;
    t.schedule = rkmi::kSchedPlain;
    t.ws = static_cast<unsigned char*>(tape->tape) + tl.off_order;
    t.ws_bytes = tape->tape_bytes - tl.off_order;
    rc = rkmi::launch_cost_ordered(
        &t, 0,
        [&](const rkmi::LaunchArgs* la, void* st) {
          return la->pilot ? p->launch(la, st) : p->taped(la, tape, st);
        },
        stream);
  } else if (opt && opt->cost_order) {
    const int64_t base = p->workspace(method, a.schedule, n);
    if (base < 0) return fail(RK_EHIP, "could not query the current device");
    rc = rkmi::launch_cost_ordered(&a, (size_t)base, p->launch, stream);
  } else {
    rc = tape ? p->taped(&a, tape, stream) : p->launch(&a, stream);
  }
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
  p->gershgorin = true;
  p->n_eq = 2;
  p->n_param = 1;
  p->n_theta = 1;
  p->launch = rkmi_vdp_launch;
  p->host = rkmi_vdp_host;
  p->workspace = rkmi_vdp_workspace;
  p->taped = rkmi_vdp_taped;
  p->taped_host = rkmi_vdp_taped_host;
  p->adjoint = rkmi_vdp_adjoint;
  p->adjoint_host = rkmi_vdp_adjoint_host;
  *out = p;
  return RK_OK;
}

int rk_problem_create_pleiades(rk_problem* out) {
  g_err.clear();
  if (!out) return fail(RK_EINVAL, "out is NULL");
  *out = nullptr;
  rk_problem p = new (std::nothrow) rk_problem_s();
  if (!p) return fail(RK_ENOMEM, "out of host memory");
  p->kind = kPleiades;
  p->n_eq = 28;
  p->n_param = 0;
  p->n_theta = 0;
  p->launch = rkmi_pleiades_launch;
  p->host = rkmi_pleiades_host;
  p->workspace = rkmi_pleiades_workspace;
  *out = p;
  return RK_OK;
}

}  // extern "C"

namespace {

// A compiled mass-action network, isothermal (thermo = NULL) or with the
// energy equation (thermo = [u0 | cv0 | cv1], n_sp each).
int create_mass_action(const rk_mech_desc* d, const double* thermo, rk_problem* out) {
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
  int hit_index = -1;
  for (int e = 0; e < rkmi::kGenRegistrySize; ++e) {
    const rkmi::GenEntry& E = rkmi::kGenRegistry[e];
    if (E.thermal != (thermo ? 1 : 0)) continue;
    if (E.n_sp == d->n_sp && E.n_rx == d->n_rx &&
        !std::memcmp(E.reac, d->reac, sizeof(int32_t) * 2 * d->n_rx) &&
        !std::memcmp(E.prod, d->prod, sizeof(int32_t) * 2 * d->n_rx)) {
      hit = &E;
      hit_index = e;
      break;
    }
  }
  if (!hit)
    return fail(RK_EUNSUPPORTED,
                "no compiled right-hand side for this %d-species / %d-reaction topology%s; "
                "generate it with the package code generator and rebuild",
                d->n_sp, d->n_rx, thermo ? " with the energy equation" : "");
  rk_problem p = new (std::nothrow) rk_problem_s();
  if (!p) return fail(RK_ENOMEM, "out of host memory");
  p->kind = thermo ? kMassActionThermal : kMassAction;
  p->gershgorin = !thermo && d->n_sp <= 16;
  p->n_eq = d->n_sp + (thermo ? 1 : 0);
  p->n_param = thermo ? 1 : 2;
  p->n_theta = thermo ? 0 : d->n_rx;
  p->n_rx = d->n_rx;
  p->launch = hit->launch;
  p->host = hit->host;
  p->workspace = hit->workspace;
  p->taped = hit->taped;
  p->taped_host = hit->taped_host;
  p->adjoint = hit->adjoint;
  p->adjoint_host = hit->adjoint_host;
  p->gen_index = hit_index;
  const int nr = d->n_rx, ns = d->n_sp;
  p->host_prm.resize(4 * nr + (thermo ? 5 : 2) * ns);
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
  if (thermo)
    for (int k = 0; k < 3 * ns; ++k) p->host_prm[4 * nr + 2 * ns + k] = thermo[k];
  *out = p;
  return RK_OK;
}

}  // namespace

extern "C" {

int rk_problem_create_mass_action(const rk_mech_desc* d, rk_problem* out) {
  g_err.clear();
  return create_mass_action(d, nullptr, out);
}

int rk_problem_create_mass_action_thermal(const rk_mech_desc* d, const double* u0,
                                          const double* cv0, const double* cv1,
                                          rk_problem* out) {
  g_err.clear();
  if (!d || !u0 || !cv0 || !cv1 || !out) {
    if (out) *out = nullptr;
    return fail(RK_EINVAL, "desc, u0, cv0, cv1 and out are required");
  }
  if (d->n_sp <= 0 || d->n_sp > 4096) return fail(RK_EINVAL, "bad n_sp");
  std::vector<double> th(3 * (size_t)d->n_sp);
  for (int k = 0; k < d->n_sp; ++k) {
    th[k] = u0[k];
    th[d->n_sp + k] = cv0[k];
    th[2 * d->n_sp + k] = cv1[k];
    if (!std::isfinite(u0[k]) || !(cv0[k] > 0.0) || !std::isfinite(cv1[k]))
      return fail(RK_EINVAL, "species %d has invalid thermodynamic data", k);
  }
  return create_mass_action(d, th.data(), out);
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
  if (schedule < rkmi::kSchedAuto || schedule > rkmi::kSchedGroup) return 0;
  const int64_t b = p->workspace(method == RK_METHOD_RKCK ? rkmi::kMethodRkck : rkmi::kMethodRkc,
                                 schedule, n_sys);
  if (b < 0) {
    fail(RK_EHIP, "could not query the current device");
    return 0;
  }
  if (opt && opt->cost_order) return rkmi::order_layout((size_t)b, n_sys).bytes;
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

}  // extern "C"

// ----------------------------------------------------------------------------
// Workspace of the allocation-free RKC entry point: one array per device,
// loaded with the code object and held until the process ends.  Host code
// never uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) unsigned char scratch[RK_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`.
int scratch_address(void** out) {
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(RK_EHIP, "no usable current HIP device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(RK_EHIP, "no device address for the scratch array on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RK_OK;
}

}  // namespace

extern "C" {

int rk_integrate_rkc_noalloc(rk_problem p, int64_t n_sys, const double* y0, double* y1,
                             const double* g, double t0, double t1, double rtol, double atol,
                             int32_t* status, int32_t* stats, const rk_options* opt,
                             void* stream) {
  g_err.clear();
  if (!p) return fail(RK_EINVAL, "problem handle is NULL");
  if (n_sys <= 0 || !(t1 > t0))   // nothing to size; integrate() checks and handles these
    return integrate(rkmi::kMethodRkc, p, n_sys, y0, y1, g, t0, t1, rtol, atol, status, stats,
                     nullptr, 0, opt, stream, nullptr, nullptr, false, true);
  const size_t need = rk_workspace_bytes(p, RK_METHOD_RKC, n_sys, opt);
  if (!g_err.empty()) return RK_EHIP;
  if (need > (size_t)RK_SCRATCH_BYTES)
    return fail(RK_EWORKSPACE, "this call needs %zu bytes of workspace; the allocation-free "
                "entry point has %zu (use rk_integrate_rkc with a workspace of that size)", need,
                (size_t)RK_SCRATCH_BYTES);
  void* ws = nullptr;
  int rc;
  if (need && (rc = scratch_address(&ws))) return rc;
  return integrate(rkmi::kMethodRkc, p, n_sys, y0, y1, g, t0, t1, rtol, atol, status, stats, ws,
                   need, opt, stream, nullptr, nullptr, false, true);
}

size_t rk_tape_bytes(rk_problem p, int64_t n_sys, int64_t max_accepted, int32_t ckpt_every) {
  g_err.clear();
  if (!p || n_sys < 0 || max_accepted < 0 || ckpt_every < 1) return 0;
  return rkmi::tape_layout(n_sys, max_accepted, ckpt_every, p->n_eq).bytes;
}

int rk_integrate_rkc_taped(rk_problem p, int64_t n_sys, const double* y0, double* y1,
                           const double* g, double t0, double t1, double rtol, double atol,
                           int32_t* status, int32_t* stats, void* tape, size_t tape_bytes,
                           int64_t max_accepted, int32_t ckpt_every, const rk_options* opt,
                           void* stream) {
  const rkmi::TapeArgs t{tape, tape_bytes, max_accepted, ckpt_every};
  return integrate(rkmi::kMethodRkc, p, n_sys, y0, y1, g, t0, t1, rtol, atol, status, stats,
                   nullptr, 0, opt, stream, &t);
}

size_t rk_carry_rows(rk_problem p) {
  g_err.clear();
  return p ? (size_t)(rkmi::kCarryRows + p->n_eq) : 0;
}

int rk_integrate_rkck_carry(rk_problem p, int64_t n_sys, const double* y0, double* y1,
                            const double* g, double t0, double t1, double rtol, double atol,
                            int32_t* status, int32_t* stats, double* carry, void* ws,
                            size_t ws_bytes, const rk_options* opt, void* stream) {
  return integrate(rkmi::kMethodRkck, p, n_sys, y0, y1, g, t0, t1, rtol, atol, status, stats, ws,
                   ws_bytes, opt, stream, nullptr, carry, true);
}

int rk_integrate_rkc_carry(rk_problem p, int64_t n_sys, const double* y0, double* y1,
                           const double* g, double t0, double t1, double rtol, double atol,
                           int32_t* status, int32_t* stats, double* carry, void* ws,
                           size_t ws_bytes, const rk_options* opt, void* stream) {
  return integrate(rkmi::kMethodRkc, p, n_sys, y0, y1, g, t0, t1, rtol, atol, status, stats, ws,
                   ws_bytes, opt, stream, nullptr, carry, true);
}

int rk_integrate_rkck_taped(rk_problem p, int64_t n_sys, const double* y0, double* y1,
                            const double* g, double t0, double t1, double rtol, double atol,
                            int32_t* status, int32_t* stats, void* tape, size_t tape_bytes,
                            int64_t max_accepted, int32_t ckpt_every, const rk_options* opt,
                            void* stream) {
  const rkmi::TapeArgs t{tape, tape_bytes, max_accepted, ckpt_every};
  return integrate(rkmi::kMethodRkck, p, n_sys, y0, y1, g, t0, t1, rtol, atol, status, stats,
                   nullptr, 0, opt, stream, &t);
}

}  // extern "C"

namespace {

// Adjoint workspace: per 64 systems one block of per-lane columns (RKC:
// max_stages stage records of N + 4 doubles; RKCK: the six stage arguments and
// their adjoints, 12 N doubles), plus ckpt_every step-start states; then the
// order in which the reverse sweep hands systems to lanes (order_layout).
size_t adjoint_ws_bytes(int method, rk_problem p, int64_t n_sys, int32_t max_stages,
                        int32_t ckpt_every) {
  if (!p || n_sys <= 0 || ckpt_every < 1) return 0;
  if (method == rkmi::kMethodRkc && max_stages < 2) return 0;
  const int64_t blocks = (n_sys + rkmi::kLdsStride - 1) / rkmi::kLdsStride;
  const int64_t per = method == rkmi::kMethodRkck ? 12 * (int64_t)p->n_eq
                                                  : (int64_t)max_stages * (p->n_eq + 4);
  const int64_t rows = per + (int64_t)ckpt_every * p->n_eq;
  return rkmi::order_layout((size_t)(blocks * rows * rkmi::kLdsStride * (int64_t)sizeof(double)),
                            n_sys)
      .bytes;
}

int adjoint(int method, rk_problem p, int64_t n_sys, const double* g, const void* tape,
            size_t tape_bytes, int64_t max_accepted, int32_t ckpt_every, int32_t max_stages,
            const double* dL_dy1, double* dL_dy0, double* dL_dtheta, int32_t* status, void* ws,
            size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!p) return fail(RK_EINVAL, "problem handle is NULL");
  if (!p->adjoint)
    return fail(RK_EUNSUPPORTED, "the adjoint is not compiled for this problem (systems of "
                "more than 16 unknowns keep their vectors in workspace columns)");
  if (n_sys < 0) return fail(RK_EINVAL, "n_sys = %lld is negative", (long long)n_sys);
  if (ckpt_every < 1 || max_accepted < 0 || (method == rkmi::kMethodRkc && max_stages < 2))
    return fail(RK_EINVAL, "need ckpt_every >= 1, max_accepted >= 0 and (RKC) max_stages >= 2");
  if (n_sys == 0) return RK_OK;
  int rc;
  if ((rc = check_device_ptr(g, 8, "g", p->n_param == 0))) return rc;
  if ((rc = check_device_ptr(tape, 256, "tape", false))) return rc;
  if ((rc = check_device_ptr(dL_dy1, 8, "dL_dy1", false))) return rc;
  if ((rc = check_device_ptr(dL_dy0, 8, "dL_dy0", false))) return rc;
  if ((rc = check_device_ptr(dL_dtheta, 8, "dL_dtheta", true))) return rc;
  if ((rc = check_device_ptr(status, 4, "status", true))) return rc;
  if ((rc = check_device_ptr(ws, 8, "ws", false))) return rc;
  const size_t tneed = rkmi::tape_layout(n_sys, max_accepted, ckpt_every, p->n_eq).bytes;
  if (tape_bytes < tneed)
    return fail(RK_EINVAL, "tape of %zu bytes is smaller than its layout (%zu)", tape_bytes, tneed);
  const size_t wneed = adjoint_ws_bytes(method, p, n_sys, max_stages, ckpt_every);
  if (ws_bytes < wneed)
    return fail(RK_EWORKSPACE, "workspace of %zu bytes is too small (%zu needed)", ws_bytes, wneed);
  rkmi::AdjointArgs a{};
  a.method = method;
  a.n = n_sys;
  a.g = g;
  a.tape = rkmi::TapeArgs{const_cast<void*>(tape), tape_bytes, max_accepted, ckpt_every};
  a.max_stages = max_stages;
  a.w = dL_dy1;
  a.dy0 = dL_dy0;
  a.dth = dL_dtheta;
  a.status = status;
  a.ws = ws;
  a.ws_bytes = ws_bytes;
  if ((rc = problem_device_data(p, &a.prm))) return rc;
  rc = p->adjoint(&a, stream);
  if (rc) return fail(RK_EHIP, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
  return RK_OK;
}

}  // namespace

extern "C" {

size_t rk_adjoint_workspace_bytes(rk_problem p, int64_t n_sys, int32_t max_stages,
                                  int32_t ckpt_every) {
  g_err.clear();
  return adjoint_ws_bytes(rkmi::kMethodRkc, p, n_sys, max_stages, ckpt_every);
}

size_t rk_adjoint_rkck_workspace_bytes(rk_problem p, int64_t n_sys, int32_t ckpt_every) {
  g_err.clear();
  return adjoint_ws_bytes(rkmi::kMethodRkck, p, n_sys, 0, ckpt_every);
}

int rk_adjoint_rkc(rk_problem p, int64_t n_sys, const double* g, const void* tape,
                   size_t tape_bytes, int64_t max_accepted, int32_t ckpt_every,
                   int32_t max_stages, const double* dL_dy1, double* dL_dy0, double* dL_dtheta,
                   int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  return adjoint(rkmi::kMethodRkc, p, n_sys, g, tape, tape_bytes, max_accepted, ckpt_every,
                 max_stages, dL_dy1, dL_dy0, dL_dtheta, status, ws, ws_bytes, stream);
}

int rk_adjoint_rkck(rk_problem p, int64_t n_sys, const double* g, const void* tape,
                    size_t tape_bytes, int64_t max_accepted, int32_t ckpt_every,
                    const double* dL_dy1, double* dL_dy0, double* dL_dtheta, int32_t* status,
                    void* ws, size_t ws_bytes, void* stream) {
  return adjoint(rkmi::kMethodRkck, p, n_sys, g, tape, tape_bytes, max_accepted, ckpt_every, 0,
                 dL_dy1, dL_dy0, dL_dtheta, status, ws, ws_bytes, stream);
}

struct rk_batch_s {
  const rkmi::BatchEntry* entry = nullptr;
  rk_problem probs[rkmi::kBatchMaxNets] = {};  // in the caller's order
  int user_to_entry[rkmi::kBatchMaxNets] = {};
  int n = 0;
  void* graph_cache = nullptr;
  std::mutex mu;
};

int rk_batch_create(const rk_problem* probs, int32_t n_prob, rk_batch* out) {
  g_err.clear();
  if (!out) return fail(RK_EINVAL, "out is NULL");
  *out = nullptr;
  if (!probs || n_prob < 1 || n_prob > rkmi::kBatchMaxNets)
    return fail(RK_EINVAL, "need 1..%d problems", rkmi::kBatchMaxNets);
  for (int k = 0; k < n_prob; ++k)
    if (!probs[k] || probs[k]->gen_index < 0)
      return fail(RK_EINVAL, "problem %d is not a compiled mass-action network", k);
  for (int e = 0; e < rkmi::kBatchRegistrySize; ++e) {
    const rkmi::BatchEntry& E = rkmi::kBatchRegistry[e];
    if (E.n_net != n_prob || !E.launch) continue;
    int map[rkmi::kBatchMaxNets];
    bool used[rkmi::kBatchMaxNets] = {};
    bool ok = true;
    for (int k = 0; k < n_prob && ok; ++k) {
      map[k] = -1;
      for (int j = 0; j < E.n_net; ++j)
        if (!used[j] && E.gen_index[j] == probs[k]->gen_index) {
          map[k] = j;
          used[j] = true;
          break;
        }
      ok = map[k] >= 0;
    }
    if (!ok) continue;
    rk_batch b = new (std::nothrow) rk_batch_s();
    if (!b) return fail(RK_ENOMEM, "out of host memory");
    b->entry = &E;
    b->n = n_prob;
    for (int k = 0; k < n_prob; ++k) {
      b->probs[k] = probs[k];
      b->user_to_entry[k] = map[k];
    }
    b->graph_cache = new (std::nothrow) rkmi::BatchGraphCache();
    if (!b->graph_cache) {
      delete b;
      return fail(RK_ENOMEM, "out of host memory");
    }
    *out = b;
    return RK_OK;
  }
  return fail(RK_EUNSUPPORTED, "no batch kernel is compiled for this set of networks");
}

void rk_batch_destroy(rk_batch b) {
  if (!b) return;
  if (b->graph_cache) b->entry->free_cache(b->graph_cache);
  delete b;
}

namespace {

// Fills the batch arguments in the compiled network order.
int batch_args(rk_batch b, const int64_t* n_sys, double* const* y, const double* const* g,
               int32_t* const* status, int32_t* const* stats, const int32_t* map, int64_t n_total,
               double t0, double dt, int32_t n_substeps, double rtol, double atol,
               const rk_options* opt, const rk_batch_schedule* sched, void* ws, size_t ws_bytes,
               bool with_pointers, rkmi::BatchArgs& a) {
  a = rkmi::BatchArgs{};
  a.mode = sched ? sched->mode : RK_BATCH_PERSISTENT;
  if (a.mode < RK_BATCH_PERSISTENT || a.mode > RK_BATCH_PLAIN_PER_NETWORK)
    return fail(RK_EUNSUPPORTED, "batch mode %d is not available", a.mode);
  if (sched)
    for (int k = 0; k < 4; ++k)
      if (sched->reserved[k]) return fail(RK_EINVAL, "rk_batch_schedule.reserved must be zero");
  a.n_net = b->n;
  a.waves_per_cu = sched ? sched->waves_per_cu : 0;
  a.use_graph = sched ? sched->use_graph : 0;
  for (int k = 0; k < rkmi::kBatchMaxNets; ++k) a.order[k] = k, a.map_net[k] = 0;
  for (int k = 0; k < b->n; ++k) {
    const int e = b->user_to_entry[k];
    if (n_sys[k] < 0 || n_sys[k] > 0x0fffffff)
      return fail(RK_EINVAL, "n_sys[%d] = %lld out of range", k, (long long)n_sys[k]);
    a.net[e].n = n_sys[k];
    a.map_net[k] = e;
    a.refill[e] = sched ? sched->refill[k] : 0;
    if (with_pointers && n_sys[k] > 0) {
      int rc;
      if ((rc = check_device_ptr(y[k], 8, "y", false))) return rc;
      if ((rc = check_device_ptr(g[k], 8, "g", false))) return rc;
      if (status && (rc = check_device_ptr(status[k], 4, "status", true))) return rc;
      if (stats && (rc = check_device_ptr(stats[k], 4, "stats", true))) return rc;
      if ((rc = problem_device_data(b->probs[k], &a.net[e].prm))) return rc;
      a.net[e].y = y[k];
      a.net[e].g = g[k];
      a.net[e].status = status ? status[k] : nullptr;
      a.net[e].stats = stats ? stats[k] : nullptr;
    }
  }
  // order: as given, else the largest networks first
  bool given = sched && sched->order[0] >= 0;
  if (given) {
    bool seen[rkmi::kBatchMaxNets] = {};
    for (int r = 0; r < b->n; ++r) {
      const int k = sched->order[r];
      if (k < 0 || k >= b->n || seen[k]) return fail(RK_EINVAL, "order is not a permutation");
      seen[k] = true;
      a.order[r] = b->user_to_entry[k];
    }
  } else {
    int idx[rkmi::kBatchMaxNets];
    for (int k = 0; k < b->n; ++k) idx[k] = k;
    for (int i = 0; i < b->n; ++i)
      for (int j = i + 1; j < b->n; ++j)
        if (b->probs[idx[j]]->n_eq > b->probs[idx[i]]->n_eq) std::swap(idx[i], idx[j]);
    for (int r = 0; r < b->n; ++r) a.order[r] = b->user_to_entry[idx[r]];
  }
  a.map = map;
  a.n_total = n_total;
  if (a.mode == RK_BATCH_PLAIN_INTERLEAVED) {
    int64_t tot = 0;
    for (int k = 0; k < b->n; ++k) tot += n_sys[k];
    if (n_total != tot) return fail(RK_EINVAL, "n_total must be the sum of n_sys");
    if (with_pointers && n_total > 0) {
      int rc;
      if ((rc = check_device_ptr(map, 4, "slot_map", false))) return rc;
    }
  }
  if (!std::isfinite(t0) || !std::isfinite(dt) || !(dt > 0.0) || n_substeps < 0)
    return fail(RK_EINVAL, "need finite t0, dt > 0 and n_substeps >= 0");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(RK_EINVAL, "rtol must be positive");
  if (!(atol >= 0.0) || !std::isfinite(atol)) return fail(RK_EINVAL, "atol must be >= 0");
  fill_ctl(a.ctl, t0, t0 + dt, rtol, atol, opt);
  a.t0 = t0;
  a.dt = dt;
  a.n_substeps = n_substeps;
  a.ws = ws;
  a.ws_bytes = ws_bytes;
  a.graph_cache = b->graph_cache;
  return RK_OK;
}

}  // namespace

size_t rk_batch_workspace_bytes(rk_batch b, const int64_t* n_sys, int64_t n_total,
                                const rk_batch_schedule* sched) {
  g_err.clear();
  if (!b || !n_sys) return 0;
  rkmi::BatchArgs a;
  if (batch_args(b, n_sys, nullptr, nullptr, nullptr, nullptr, nullptr, n_total, 0.0, 1.0, 1,
                 1e-6, 0.0, nullptr, sched, nullptr, 0, false, a))
    return 0;
  const int64_t need = b->entry->workspace(&a);
  if (need < 0) {
    fail(RK_EHIP, "could not query the current device");
    return 0;
  }
  return (size_t)need;
}

int rk_batch_integrate_rkc(rk_batch b, const int64_t* n_sys, double* const* y,
                           const double* const* g, int32_t* const* status, int32_t* const* stats,
                           double* const* carry, const int32_t* slot_map, int64_t n_total,
                           double t0, double dt, int32_t n_substeps, double rtol, double atol,
                           const rk_options* opt, const rk_batch_schedule* sched, void* ws,
                           size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!b) return fail(RK_EINVAL, "batch handle is NULL");
  if (!n_sys || !y || !g) return fail(RK_EINVAL, "n_sys, y and g are required");
  if (opt) {
    for (size_t k = 0; k < sizeof(opt->reserved) / sizeof(opt->reserved[0]); ++k)
      if (opt->reserved[k]) return fail(RK_EINVAL, "rk_options.reserved must be zero");
    if (opt->cost_order)
      return fail(RK_EUNSUPPORTED, "cost_order is not available for a batch");
    if (opt->sr_method)
      return fail(RK_EUNSUPPORTED, "sr_method is not available for a batch");
  }
  rkmi::BatchArgs a;
  int rc = batch_args(b, n_sys, y, g, status, stats, slot_map, n_total, t0, dt, n_substeps, rtol,
                      atol, opt, sched, ws, ws_bytes, true, a);
  if (rc) return rc;
  if (carry)
    for (int k = 0; k < b->n; ++k) {
      if (n_sys[k] == 0) continue;
      if ((rc = check_device_ptr(carry[k], 8, "carry", false))) return rc;
      a.net[b->user_to_entry[k]].carry = carry[k];
    }
  if ((rc = check_device_ptr(ws, 256, "ws", true))) return rc;
  std::lock_guard<std::mutex> lock(b->mu);
  rc = b->entry->launch(&a, stream);
  if (rc == rkmi::kLaunchWorkspace)
    return fail(RK_EWORKSPACE, "workspace of %zu bytes is too small (rk_batch_workspace_bytes "
                "gives the size this call needs)", ws ? ws_bytes : (size_t)0);
  if (rc == rkmi::kLaunchInvalid) return fail(RK_EINVAL, "too many systems for one launch");
  if (rc) return fail(RK_EHIP, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
  return RK_OK;
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

// As rkmi_test_host_integrate with the RKC spectral radius of sr_method.
int rkmi_test_host_integrate_sr(int32_t method, rk_problem p, int64_t n, const double* y0,
                                double* y1, const double* g, double t0, double t1, double rtol,
                                double atol, int32_t* status, int32_t* stats, int64_t max_steps,
                                int32_t sr_method) {
  g_err.clear();
  if (!p || !p->host || n < 0 || !y0 || !y1 || (p->n_param && !g) || !(t1 > t0) ||
      !(rtol > 0.0) || !(atol >= 0.0) || sr_method < 0 || sr_method > 1 ||
      (sr_method == 1 && !p->gershgorin))
    return fail(RK_EINVAL, "invalid arguments");
  rk_options o{};
  o.max_steps = max_steps;
  o.sr_method = sr_method;
  rkmi::LaunchArgs a;
  fill_args(a, method, n, y0, y1, g, t0, t1, rtol, atol, status, stats, nullptr, 0, &o);
  a.prm = p->host_prm.empty() ? nullptr : p->host_prm.data();
  return p->host(&a);
}

// As rkmi_test_host_integrate with a carried controller state (host array
// [kCarryRows + N][n], read and rewritten).
int rkmi_test_host_integrate_carry(int32_t method, rk_problem p, int64_t n, const double* y0,
                                   double* y1, const double* g, double t0, double t1,
                                   double rtol, double atol, int32_t* status, int32_t* stats,
                                   int64_t max_steps, double* carry) {
  g_err.clear();
  if (!p || !p->host || n < 0 || !y0 || !y1 || (p->n_param && !g) || !(t1 >= t0) ||
      !(rtol > 0.0) || !(atol >= 0.0) || !carry)
    return fail(RK_EINVAL, "invalid arguments");
  rk_options o{};
  o.max_steps = max_steps;
  rkmi::LaunchArgs a;
  fill_args(a, method, n, y0, y1, g, t0, t1, rtol, atol, status, stats, nullptr, 0, &o);
  a.prm = p->host_prm.empty() ? nullptr : p->host_prm.data();
  a.carry = carry;
  return p->host(&a);
}

// Test hooks, not part of the public ABI: the taped forward and the adjoint's
// per-system code run on the host over HOST arrays (tape and workspace too).
int rkmi_test_host_taped(rk_problem p, int32_t method, int64_t n, const double* y0, double* y1,
                         const double* g, double t0, double t1, double rtol, double atol,
                         int32_t* status, int32_t* stats, void* tape, size_t tape_bytes,
                         int64_t cap, int32_t K) {
  g_err.clear();
  if (!p || !p->taped_host || n < 0 || !y0 || !y1 || (p->n_param && !g) || !(t1 >= t0) ||
      !(rtol > 0.0) || !(atol >= 0.0) || !tape || K < 1 || cap < 0 ||
      (method != RK_METHOD_RKCK && method != RK_METHOD_RKC))
    return fail(RK_EINVAL, "invalid arguments");
  rkmi::LaunchArgs a;
  fill_args(a, method == RK_METHOD_RKCK ? rkmi::kMethodRkck : rkmi::kMethodRkc, n, y0, y1, g, t0,
            t1, rtol, atol, status, stats, nullptr, 0, nullptr);
  a.prm = p->host_prm.empty() ? nullptr : p->host_prm.data();
  const rkmi::TapeArgs t{tape, tape_bytes, cap, K};
  return p->taped_host(&a, &t);
}

int rkmi_test_host_adjoint(rk_problem p, int32_t method, int64_t n, const double* g, void* tape,
                           size_t tape_bytes, int64_t cap, int32_t K, int32_t max_stages,
                           const double* w, double* dy0, double* dth, int32_t* status) {
  g_err.clear();
  if (!p || !p->adjoint_host || n < 0 || !tape || !w || !dy0 ||
      (method != RK_METHOD_RKCK && method != RK_METHOD_RKC))
    return fail(RK_EINVAL, "invalid arguments");
  rkmi::AdjointArgs a{};
  a.method = method == RK_METHOD_RKCK ? rkmi::kMethodRkck : rkmi::kMethodRkc;
  a.n = n;
  a.g = g;
  a.prm = p->host_prm.empty() ? nullptr : p->host_prm.data();
  a.tape = rkmi::TapeArgs{tape, tape_bytes, cap, K};
  a.max_stages = max_stages;
  a.w = w;
  a.dy0 = dy0;
  a.dth = dth;
  a.status = status;
  return p->adjoint_host(&a);
}

}  // extern "C"
