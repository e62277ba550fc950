// rk_launch.hpp -- host-side launch plumbing shared by every compiled problem.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "rk_device.hpp"
#include "rk_types.hpp"

namespace rkmi {

enum : int { kSchedAuto = 0, kSchedPlain = 1, kSchedPersistent = 2, kSchedGroup = 3 };

// Launch error codes (mapped to RK_* by the ABI layer).
enum : int { kLaunchOk = 0, kLaunchInvalid = -1, kLaunchHip = -3, kLaunchWorkspace = -5 };

// Workspace layout: [queue head, kQueueBytes][column blocks, one per workgroup].
constexpr size_t kQueueBytes = 256;

// Idle lanes that make a wave of the persistent kernel take new systems.
constexpr int kDefaultRefill = 16;

template <int = 0>
__global__ void queue_reset_kernel(unsigned long long* queue) {
  queue[0] = 0ull;
}

// Bytes of column workspace one workgroup uses (zero for register-held systems).
template <class Prob, int Method>
constexpr size_t block_col_bytes() {
  return Prob::kColumns ? (size_t)slot_doubles<Prob, Method>() * kLdsStride * sizeof(double) : 0;
}

// Workgroups of the persistent grid: every resident slot the occupancy allows
// on every compute unit of the current device, at most one per 64 systems.
template <class Prob, int Method>
int persistent_grid(int64_t blocks, int64_t* grid) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<Prob, Method>,
                                                   kLdsStride, 0) != hipSuccess)
    return kLaunchHip;
  if (per_cu < 1) per_cu = 1;
  const int64_t g = (int64_t)cus * per_cu;
  *grid = g < blocks ? g : blocks;
  return kLaunchOk;
}

// Workspace bytes a launch needs under `schedule` (auto counts as persistent).
template <class Prob, int Method>
int64_t workspace_bytes(int schedule, int64_t n) {
  const int64_t blocks = (n + kLdsStride - 1) / kLdsStride;
  if (blocks <= 0) return 0;
  if (schedule == kSchedPlain)
    return Prob::kColumns ? (int64_t)kQueueBytes + blocks * (int64_t)block_col_bytes<Prob, Method>()
                          : 0;
  int64_t grid = 0;
  if (persistent_grid<Prob, Method>(blocks, &grid) != kLaunchOk) return -1;
  return (int64_t)kQueueBytes + grid * (int64_t)block_col_bytes<Prob, Method>();
}

template <class Prob, int Method, bool kPilot>
int launch_method(const LaunchArgs* a, hipStream_t s) {
  const int64_t blocks = (a->n + kLdsStride - 1) / kLdsStride;
  if (blocks <= 0) return kLaunchOk;
  if (blocks > 0x7fffffffLL) return kLaunchInvalid;
  const typename Prob::Params prm = a->prm;
  constexpr size_t col_bytes = block_col_bytes<Prob, Method>();
  const size_t ws_bytes = a->ws ? a->ws_bytes : 0;
  unsigned char* const ws = static_cast<unsigned char*>(a->ws);
  double* const cols = ws ? reinterpret_cast<double*>(ws + kQueueBytes) : nullptr;
  // persistent when asked, or by default when the workspace holds the queue and
  // at least one workgroup's columns
  // (the group schedule means the default one for problems without a group variant)
  const bool persistent =
      a->schedule == kSchedPersistent ||
      ((a->schedule == kSchedAuto || a->schedule == kSchedGroup) &&
       ws_bytes >= kQueueBytes + col_bytes);
  if (!persistent) {
    if (col_bytes && ws_bytes < kQueueBytes + (size_t)blocks * col_bytes) return kLaunchWorkspace;
    plain_kernel<Prob, Method, kPilot><<<dim3((unsigned)blocks), dim3(kLdsStride), 0, s>>>(
        prm, a->n, a->y0, a->y1, a->g, a->ctl, a->status, a->stats, cols, a->order, a->carry);
    return hipGetLastError() == hipSuccess ? kLaunchOk : kLaunchHip;
  }
  int64_t grid = 0;
  if (persistent_grid<Prob, Method>(blocks, &grid) != kLaunchOk) return kLaunchHip;
  if (ws_bytes < kQueueBytes + col_bytes) return kLaunchWorkspace;
  if (col_bytes) {
    // a smaller workspace runs a smaller grid
    const int64_t fit = (int64_t)((ws_bytes - kQueueBytes) / col_bytes);
    if (grid > fit) grid = fit;
  }
  unsigned long long* queue = reinterpret_cast<unsigned long long*>(ws);
  queue_reset_kernel<><<<1, 1, 0, s>>>(queue);
  persistent_kernel<Prob, Method, kPilot><<<dim3((unsigned)grid), dim3(kLdsStride), 0, s>>>(
      prm, a->n, a->y0, a->y1, a->g, a->ctl, a->status, a->stats, queue, cols, a->order,
      a->carry);
  return hipGetLastError() == hipSuccess ? kLaunchOk : kLaunchHip;
}

template <class Prob>
int launch(const LaunchArgs* a, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if constexpr (HasGershgorin<Prob>::value && !SigmaFromGershgorin<Prob>::value) {
    if (a->method == kMethodRkc && a->ctl.sr_method == kSrGershgorin)
      return a->pilot ? launch_method<WithGershgorin<Prob>, kMethodRkc, true>(a, s)
                      : launch_method<WithGershgorin<Prob>, kMethodRkc, false>(a, s);
  }
  if (a->pilot)
    return a->method == kMethodRkck ? launch_method<Prob, kMethodRkck, true>(a, s)
                                    : launch_method<Prob, kMethodRkc, true>(a, s);
  return a->method == kMethodRkck ? launch_method<Prob, kMethodRkck, false>(a, s)
                                  : launch_method<Prob, kMethodRkc, false>(a, s);
}

template <class Prob>
int64_t workspace(int method, int schedule, int64_t n) {
  return method == kMethodRkck ? workspace_bytes<Prob, kMethodRkck>(schedule, n)
                               : workspace_bytes<Prob, kMethodRkc>(schedule, n);
}

// The per-system code of the kernels, run on the host for every system (test
// hook: the same source compiled for the CPU; each system is independent, so
// the schedule does not change any result).
template <class Prob>
int host_run(const LaunchArgs* a) {
  std::vector<double> slot((size_t)(slot_doubles<Prob, kMethodRkck>() >
                                            slot_doubles<Prob, kMethodRkc>()
                                        ? slot_doubles<Prob, kMethodRkck>()
                                        : slot_doubles<Prob, kMethodRkc>()) *
                               kLdsStride +
                           1);
  for (int64_t i = 0; i < a->n; ++i) {
    if constexpr (HasGershgorin<Prob>::value && !SigmaFromGershgorin<Prob>::value) {
      if (a->method == kMethodRkc && a->ctl.sr_method == kSrGershgorin) {
        integrate_system<WithGershgorin<Prob>, kMethodRkc>(a->prm, a->n, i, a->y0, a->y1, a->g,
                                                           a->ctl, a->status, a->stats,
                                                           slot.data(), a->carry);
        continue;
      }
    }
    if (a->method == kMethodRkck)
      integrate_system<Prob, kMethodRkck>(a->prm, a->n, i, a->y0, a->y1, a->g, a->ctl, a->status,
                                          a->stats, slot.data(), a->carry);
    else
      integrate_system<Prob, kMethodRkc>(a->prm, a->n, i, a->y0, a->y1, a->g, a->ctl, a->status,
                                         a->stats, slot.data(), a->carry);
  }
  return 0;
}

}  // namespace rkmi
