// rk_launch.hpp -- host-side launch plumbing shared by every compiled problem.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "rk_device.hpp"
#include "rk_types.hpp"

namespace rkmi {

enum : int { kSchedAuto = 0, kSchedPlain = 1, kSchedPersistent = 2 };

// Bytes of workspace the persistent schedule needs (the queue head).
constexpr size_t kQueueBytes = 256;

// Idle lanes that make a wave of the persistent kernel take new systems.
constexpr int kDefaultRefill = 16;

template <int = 0>
__global__ void queue_reset_kernel(unsigned long long* queue) {
  queue[0] = 0ull;
}

template <class Prob, int Method>
int launch_method(const LaunchArgs* a, hipStream_t s) {
  const int64_t blocks = (a->n + kLdsStride - 1) / kLdsStride;
  if (blocks <= 0) return 0;
  if (blocks > 0x7fffffffLL) return -1;
  const typename Prob::Params prm = a->prm;
  const bool persistent = a->schedule != kSchedPlain && a->ws && a->ws_bytes >= kQueueBytes;
  if (!persistent) {
    plain_kernel<Prob, Method><<<dim3((unsigned)blocks), dim3(kLdsStride), 0, s>>>(
        prm, a->n, a->y0, a->y1, a->g, a->ctl, a->status, a->stats);
    return hipGetLastError() == hipSuccess ? 0 : -3;
  }
  // one resident wave per slot the occupancy allows on every compute unit
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<Prob, Method>,
                                                   kLdsStride, 0) != hipSuccess)
    return -3;
  if (per_cu < 1) per_cu = 1;
  int64_t grid = (int64_t)cus * per_cu;
  if (grid > blocks) grid = blocks;
  unsigned long long* queue = static_cast<unsigned long long*>(a->ws);
  queue_reset_kernel<><<<1, 1, 0, s>>>(queue);
  persistent_kernel<Prob, Method><<<dim3((unsigned)grid), dim3(kLdsStride), 0, s>>>(
      prm, a->n, a->y0, a->y1, a->g, a->ctl, a->status, a->stats, queue);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class Prob>
int launch(const LaunchArgs* a, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  return a->method == kMethodRkck ? launch_method<Prob, kMethodRkck>(a, s)
                                  : launch_method<Prob, kMethodRkc>(a, s);
}

// The per-system code of the kernels, run on the host for every system (test
// hook: the same source compiled for the CPU; each system is independent, so
// the schedule does not change any result).
template <class Prob>
int host_run(const LaunchArgs* a) {
  std::vector<double> slot((Prob::kLaneDoubles + Prob::N) * kLdsStride);
  for (int64_t i = 0; i < a->n; ++i) {
    if (a->method == kMethodRkck)
      integrate_system<Prob, kMethodRkck>(a->prm, a->n, i, a->y0, a->y1, a->g, a->ctl, a->status,
                                          a->stats, slot.data());
    else
      integrate_system<Prob, kMethodRkc>(a->prm, a->n, i, a->y0, a->y1, a->g, a->ctl, a->status,
                                         a->stats, slot.data());
  }
  return 0;
}

}  // namespace rkmi
