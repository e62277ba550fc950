// rk_types.hpp -- plain host/device types shared by the launch code and the
// registry of compiled networks (no HIP headers: the registry is host C++).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace rkmi {

enum : int { kMethodRkck = 0, kMethodRkc = 1 };

// Launch-uniform integration controls, formed on the host.
struct Ctl {
  double t0, t1;
  double rtol, atol;
  double hmax;        // |t1 - t0|
  double hmin_rkc;    // 10 UROUND max(|t0|, hmax)
  double delta;       // RKCK scale offset atol / rtol (or TINY)
  int64_t max_steps;  // attempts per system
  int mmax;           // RKC stage cap round(sqrt(rtol / (10 UROUND))), >= 2
  int sr_period;      // spectral radius every sr_period accepted steps (25)
  int sr_itmax;       // power-method iterations (50)
  int refill;         // persistent schedule: idle lanes that trigger a refill (1..64)
};

// Arguments of one integration launch (device pointers, launch-uniform controls).
struct LaunchArgs {
  int method;            // kMethodRkck | kMethodRkc
  int schedule;          // kSchedAuto | kSchedPlain | kSchedPersistent
  int64_t n;             // systems
  const double* y0;      // [N][n]
  double* y1;            // [N][n]
  const double* g;       // [P][n]
  const double* prm;     // uniform problem data on the device (may be null)
  Ctl ctl;
  int32_t* status;       // [n] or null
  int32_t* stats;        // [kNStats][n] or null
  void* ws;              // workspace (may be null)
  size_t ws_bytes;
};

// Enqueues the integration on the stream (a hipStream_t); 0 on success.
typedef int (*launch_fn)(const LaunchArgs*, void* stream);

// Runs the per-system code of the kernels on the host over host arrays (a
// test hook that checks the kernels' arithmetic on the CPU); 0 on success.
typedef int (*host_fn)(const LaunchArgs*);

// Workspace bytes a launch of `method` over n systems needs under `schedule`
// (auto counts as persistent); negative if the device cannot be queried.
typedef int64_t (*workspace_fn)(int method, int schedule, int64_t n);

// Compiled network: the topology it was generated for and its launchers.
struct GenEntry {
  int n_sp;
  int n_rx;
  const int32_t* reac;   // [n_rx][2]
  const int32_t* prod;   // [n_rx][2]
  launch_fn launch;
  host_fn host;
  workspace_fn workspace;
};

}  // namespace rkmi
