// rk_launch.hpp -- host-side launch plumbing shared by every compiled problem.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rk_device.hpp"
#include "rk_types.hpp"

namespace rkmi {

constexpr int kPlainBlock = 64;

template <class Prob>
int launch_plain(const LaunchArgs* a, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t blocks = (a->n + kPlainBlock - 1) / kPlainBlock;
  if (blocks <= 0) return 0;
  if (blocks > 0x7fffffffLL) return -1;
  const dim3 grid((unsigned)blocks), block(kPlainBlock);
  const typename Prob::Params prm = a->prm;
  if (a->method == kMethodRkck)
    plain_kernel<Prob, kMethodRkck><<<grid, block, 0, s>>>(prm, a->n, a->y0, a->y1, a->g, a->ctl,
                                                           a->status, a->stats);
  else
    plain_kernel<Prob, kMethodRkc><<<grid, block, 0, s>>>(prm, a->n, a->y0, a->y1, a->g, a->ctl,
                                                          a->status, a->stats);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// The per-system code of plain_kernel, run on the host for every system
// (test hook: the same source compiled for the CPU).
template <class Prob>
int host_run(const LaunchArgs* a) {
  constexpr int N = Prob::N;
  const typename Prob::Params prm = a->prm;
  for (int64_t i = 0; i < a->n; ++i) {
    typename Prob::Lane L;
    Prob::init(L, prm, a->g, i, a->n);
    double y[N];
    for (int k = 0; k < N; ++k) y[k] = a->y0[(int64_t)k * a->n + i];
    int32_t st[kNStats];
    const int32_t s = (a->method == kMethodRkck) ? rkck_integrate<Prob>(L, prm, a->ctl, y, st)
                                                 : rkc_integrate<Prob>(L, prm, a->ctl, y, st);
    for (int k = 0; k < N; ++k) a->y1[(int64_t)k * a->n + i] = y[k];
    if (a->status) a->status[i] = s;
    if (a->stats)
      for (int r = 0; r < kNStats; ++r) a->stats[(int64_t)r * a->n + i] = st[r];
  }
  return 0;
}

}  // namespace rkmi
