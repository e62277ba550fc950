// rk_types.hpp -- plain host/device types shared by the launch code and the
// registry of compiled networks (no HIP headers: the registry is host C++).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace rkmi {

enum : int { kMethodRkck = 0, kMethodRkc = 1 };
// RKC spectral radius: the nonlinear power method (Appendix) or the Gershgorin
// bound of the analytic Jacobian (problems with Prob::kGershgorin)
enum : int { kSrPower = 0, kSrGershgorin = 1 };

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
  int sr_method;      // kSrPower | kSrGershgorin
  int refill;         // persistent schedule: idle lanes that trigger a refill (1..64)
  int align;          // group schedule: a group at its error phase waits while another
                      // group of the wave is 1..align evaluations from its own (0: never)
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
  const int32_t* order;  // [n] queue position -> system index, or null (position = index)
  int pilot;             // nonzero: a cost-order pilot (the same kernels under their own
                         // names, so a profile tells the two passes apart)
  double* carry;         // [kCarryRows + N][n] controller state carried between calls, or null
};

// Enqueues the integration on the stream (a hipStream_t); 0 on success.
typedef int (*launch_fn)(const LaunchArgs*, void* stream);

// Runs the per-system code of the kernels on the host over host arrays (a
// test hook that checks the kernels' arithmetic on the CPU); 0 on success.
typedef int (*host_fn)(const LaunchArgs*);

// Workspace bytes a launch of `method` over n systems needs under `schedule`
// (auto counts as persistent); negative if the device cannot be queried.
typedef int64_t (*workspace_fn)(int method, int schedule, int64_t n);

// Tape of an RKC integration for the discrete adjoint: per system the number
// of accepted steps, each step's (h, s), and the state every K accepted steps.
struct TapeArgs {
  void* tape;
  size_t tape_bytes;
  int64_t cap;           // accepted steps a system can record
  int32_t K;             // checkpoint period (accepted steps)
};

// Arguments of one adjoint launch (device pointers).
struct AdjointArgs {
  int method;            // kMethodRkck | kMethodRkc (the method of the taped forward call)
  int64_t n;
  const double* g;       // [P][n]
  const double* prm;     // uniform problem data
  TapeArgs tape;
  int32_t max_stages;    // RKC: bound on the recorded stage counts
  const double* w;       // [N][n] dL/dy(t1)
  double* dy0;           // [N][n] dL/dy(t0)
  double* dth;           // [n_theta][n] per-system dL/dtheta
  int32_t* status;       // [n] or null
  void* ws;
  size_t ws_bytes;
};

typedef int (*taped_fn)(const LaunchArgs*, const TapeArgs*, void* stream);
typedef int (*taped_host_fn)(const LaunchArgs*, const TapeArgs*);
typedef int (*adjoint_fn)(const AdjointArgs*, void* stream);
typedef int (*adjoint_host_fn)(const AdjointArgs*);

// Compiled network: the topology it was generated for and its launchers.
struct GenEntry {
  int n_sp;
  int n_rx;
  const int32_t* reac;   // [n_rx][2]
  const int32_t* prod;   // [n_rx][2]
  launch_fn launch;
  host_fn host;
  workspace_fn workspace;
  taped_fn taped;                 // null where the adjoint is not compiled
  taped_host_fn taped_host;
  adjoint_fn adjoint;
  adjoint_host_fn adjoint_host;
  int thermal;                    // 1: compiled with the energy equation (state T, Y)
};

// Ragged batch of several compiled networks (rk_batch.hpp).
enum : int { kBatchPersistent = 0, kBatchInterleaved = 1, kBatchPerNet = 2 };
constexpr int kBatchMaxNets = 4;

struct BatchNetArgs {
  const double* prm;   // the network's uniform data on the device
  int64_t n;
  double* y;           // [N][n], in place
  const double* g;     // [2][n]
  int32_t* status;     // [n] or null
  int32_t* stats;      // [kNStats][n] or null
  double* carry;       // [kCarryRows + N][n] carried controller state, or null (restart)
};

struct BatchArgs {
  int32_t mode;                     // kBatchPersistent | kBatchInterleaved | kBatchPerNet
  int32_t n_net;
  BatchNetArgs net[kBatchMaxNets];  // in the compiled batch's network order
  int32_t order[kBatchMaxNets];     // persistent: networks in the order waves take them
  int32_t refill[kBatchMaxNets];    // persistent: refill threshold per network
  int32_t waves_per_cu;             // persistent: 0 = occupancy limit
  const int32_t* map;               // interleaved: [n_total] (network << 28 | index)
  int32_t map_net[kBatchMaxNets];   // interleaved: network of the map's code k
  int64_t n_total;
  Ctl ctl;                          // tolerances and limits; the launcher sets the interval
  double t0, dt;
  int32_t n_substeps;
  int32_t use_graph;                // capture the substeps in one HIP graph
  void* ws;
  size_t ws_bytes;
  void* graph_cache;                // the batch handle's cached graph (owned by the handle)
};

typedef int (*batch_fn)(const BatchArgs*, void* stream);
typedef int64_t (*batch_ws_fn)(const BatchArgs*);
typedef void (*batch_free_fn)(void* graph_cache);

// Compiled batch kernel: the networks it mixes (rows of the network registry).
struct BatchEntry {
  int n_net;
  int gen_index[kBatchMaxNets];
  batch_fn launch;
  batch_ws_fn workspace;
  batch_free_fn free_cache;
};

}  // namespace rkmi
