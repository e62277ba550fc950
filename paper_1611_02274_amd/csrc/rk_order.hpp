// rk_order.hpp -- cost-ordered hand-out of systems to lanes.
//
// A wave runs its lanes in lockstep, so it takes as long as its most
// expensive system, and the grid takes as long as its last wave; systems of
// one workload differ several-fold in their number of steps.  The cost order
// first integrates every system with both tolerances loosened (a pilot whose
// only output is each system's count of attempted steps), then hands the
// systems out in decreasing order of that count: lanes of a wave get systems
// of similar cost, and the most expensive systems start first.  The pilot's
// count ranks the systems' costs at the real tolerance closely (the step count
// of an adaptive method of order p grows like tol^(-1/(p+1)) with the same
// trajectory-dependent factor), and it costs a few per cent of the
// integration.  Each system's integration does not depend on the lane that
// runs it, so results are unchanged.
//
// The order is a counting sort on the device: histogram of the counts
// (clamped to kOrderBuckets - 1), exclusive scan in decreasing count order,
// scatter.  Systems with equal counts keep no particular order.  Every kernel
// here writes memory with vector stores and clears with a kernel, so the
// sequence can be captured in a HIP graph.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rk_device.hpp"
#include "rk_types.hpp"

namespace rkmi {

constexpr int kOrderBuckets = 4096;
constexpr int kOrderScanThreads = 256;
constexpr int kOrderPerThread = kOrderBuckets / kOrderScanThreads;
// The pilot runs at rtol * kPilotLoosen (atol scaled alike), at most
// kPilotRtolMax (and never tighter than the integration itself), and stops a
// system after kPilotMaxAttempts attempts: the costliest systems then share
// the top bucket (they start first either way), and no wave of the pilot
// waits long for one slow system.
constexpr double kPilotLoosen = 1.0e5;
constexpr double kPilotRtolMax = 1.0e-3;
constexpr int64_t kPilotMaxAttempts = 128;

constexpr size_t order_align(size_t b) { return (b + 255) / 256 * 256; }

// Workspace of the cost order, after the integration's own workspace:
// [pilot statistics kNStats x n int32][order n int32][histogram][offsets].
struct OrderLayout {
  size_t stats, order, hist, offs, bytes;
};

inline OrderLayout order_layout(size_t base_bytes, int64_t n) {
  OrderLayout L;
  L.stats = order_align(base_bytes);
  L.order = L.stats + order_align((size_t)kNStats * (size_t)n * sizeof(int32_t));
  L.hist = L.order + order_align((size_t)n * sizeof(int32_t));
  L.offs = L.hist + order_align(kOrderBuckets * sizeof(int32_t));
  L.bytes = L.offs + order_align(kOrderBuckets * sizeof(int32_t));
  return L;
}

// The pilot's controls: both tolerances scaled by the same factor, so the
// RKCK scale offset atol / rtol is unchanged; the RKC stage cap follows rtol.
inline Ctl pilot_ctl(const Ctl& c) {
  Ctl p = c;
  double r = c.rtol * kPilotLoosen;
  if (r > kPilotRtolMax) r = c.rtol > kPilotRtolMax ? c.rtol : kPilotRtolMax;
  const double f = r / c.rtol;
  p.rtol = r;
  p.atol = c.atol * f;
  const int mmax = (int)round(sqrt(r / (10.0 * kUround)));
  p.mmax = mmax < 2 ? 2 : mmax;
  if (p.max_steps > kPilotMaxAttempts) p.max_steps = kPilotMaxAttempts;
  return p;
}

template <int = 0>
__global__ void order_clear_kernel(int32_t* __restrict__ hist) {
  for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) hist[b] = 0;
}

// Bucket of system i: its pilot's attempted steps (accepted + rejected),
// clamped to the histogram.
__device__ inline int order_bucket(const int32_t* __restrict__ pstats, int64_t n, int64_t i) {
  const int64_t c = (int64_t)pstats[(int64_t)kStAccept * n + i] + pstats[(int64_t)kStReject * n + i];
  return c < 0 ? 0 : (c >= kOrderBuckets ? kOrderBuckets - 1 : (int)c);
}

// Systems per workgroup of the histogram and scatter kernels: each workgroup
// counts its chunk in LDS first, so a bucket takes one global atomic per
// workgroup rather than one per system.
constexpr int kOrderChunkThreads = 256;
constexpr int kOrderChunkPerThread = 16;
constexpr int kOrderChunk = kOrderChunkThreads * kOrderChunkPerThread;

template <int = 0>
__global__ __launch_bounds__(kOrderChunkThreads) void order_hist_kernel(
    const int32_t* __restrict__ pstats, int64_t n, int32_t* __restrict__ hist) {
  __shared__ int32_t cnt[kOrderBuckets];
  for (int b = threadIdx.x; b < kOrderBuckets; b += kOrderChunkThreads) cnt[b] = 0;
  __syncthreads();
  const int64_t first = (int64_t)blockIdx.x * kOrderChunk;
  for (int k = 0; k < kOrderChunkPerThread; ++k) {
    const int64_t i = first + (int64_t)k * kOrderChunkThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[order_bucket(pstats, n, i)], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kOrderBuckets; b += kOrderChunkThreads)
    if (cnt[b]) atomicAdd(&hist[b], cnt[b]);
}

// offs[b] = number of systems whose bucket is above b (one workgroup).
template <int = 0>
__global__ __launch_bounds__(kOrderScanThreads) void order_scan_kernel(
    const int32_t* __restrict__ hist, int32_t* __restrict__ offs) {
  __shared__ int32_t part[kOrderScanThreads];
  const int t = threadIdx.x;
  // thread t owns ranks t * kOrderPerThread .. + kOrderPerThread - 1, rank
  // r being bucket kOrderBuckets - 1 - r
  int32_t sum = 0;
  for (int k = 0; k < kOrderPerThread; ++k) sum += hist[kOrderBuckets - 1 - (t * kOrderPerThread + k)];
  part[t] = sum;
  __syncthreads();
  for (int d = 1; d < kOrderScanThreads; d <<= 1) {   // inclusive scan of the parts
    const int32_t v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = part[t] - sum;
  for (int k = 0; k < kOrderPerThread; ++k) {
    const int b = kOrderBuckets - 1 - (t * kOrderPerThread + k);
    offs[b] = run;
    run += hist[b];
  }
}

// Each workgroup ranks its chunk's systems within their buckets in LDS,
// reserves one range per bucket from the running offsets, and writes the
// systems' indices there.
template <int = 0>
__global__ __launch_bounds__(kOrderChunkThreads) void order_scatter_kernel(
    const int32_t* __restrict__ pstats, int64_t n, int32_t* __restrict__ offs,
    int32_t* __restrict__ order) {
  __shared__ int32_t cnt[kOrderBuckets];
  __shared__ int32_t base[kOrderBuckets];
  for (int b = threadIdx.x; b < kOrderBuckets; b += kOrderChunkThreads) cnt[b] = 0;
  __syncthreads();
  const int64_t first = (int64_t)blockIdx.x * kOrderChunk;
  int bucket[kOrderChunkPerThread], rank[kOrderChunkPerThread];
#pragma unroll
  for (int k = 0; k < kOrderChunkPerThread; ++k) {
    const int64_t i = first + (int64_t)k * kOrderChunkThreads + threadIdx.x;
    bucket[k] = i < n ? order_bucket(pstats, n, i) : -1;
    rank[k] = bucket[k] >= 0 ? atomicAdd(&cnt[bucket[k]], 1) : 0;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kOrderBuckets; b += kOrderChunkThreads)
    base[b] = cnt[b] ? atomicAdd(&offs[b], cnt[b]) : 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kOrderChunkPerThread; ++k) {
    const int64_t i = first + (int64_t)k * kOrderChunkThreads + threadIdx.x;
    if (bucket[k] >= 0) order[base[bucket[k]] + rank[k]] = (int32_t)i;
  }
}

// Enqueues the pilot through `launch` (the problem's launcher), the sort,
// and the integration itself with the order map.  `a` describes the
// integration; its workspace holds the integration's own `base_bytes`
// followed by order_layout's parts.
template <class LaunchFn>
int launch_cost_ordered(const LaunchArgs* a, size_t base_bytes, LaunchFn launch, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (a->n <= 0) return kLaunchOk;
  if (a->n > 0x7fffffffLL) return kLaunchInvalid;
  const OrderLayout L = order_layout(base_bytes, a->n);
  if (!a->ws || a->ws_bytes < L.bytes) return kLaunchWorkspace;
  unsigned char* const ws = static_cast<unsigned char*>(a->ws);
  int32_t* const pstats = reinterpret_cast<int32_t*>(ws + L.stats);
  int32_t* const order = reinterpret_cast<int32_t*>(ws + L.order);
  int32_t* const hist = reinterpret_cast<int32_t*>(ws + L.hist);
  int32_t* const offs = reinterpret_cast<int32_t*>(ws + L.offs);
  LaunchArgs p = *a;
  p.y1 = nullptr;
  p.status = nullptr;
  p.stats = pstats;
  p.ctl = pilot_ctl(a->ctl);
  p.ws_bytes = base_bytes;
  p.order = nullptr;
  p.pilot = 1;
  p.carry = nullptr;    // the pilot restarts and leaves a carried state alone
  int rc = launch(&p, stream);
  if (rc) return rc;
  const unsigned chunks = (unsigned)((a->n + kOrderChunk - 1) / kOrderChunk);
  order_clear_kernel<><<<1, 256, 0, s>>>(hist);
  order_hist_kernel<><<<chunks, kOrderChunkThreads, 0, s>>>(pstats, a->n, hist);
  order_scan_kernel<><<<1, kOrderScanThreads, 0, s>>>(hist, offs);
  order_scatter_kernel<><<<chunks, kOrderChunkThreads, 0, s>>>(pstats, a->n, offs, order);
  if (hipGetLastError() != hipSuccess) return kLaunchHip;
  LaunchArgs m = *a;
  m.ws_bytes = base_bytes;
  m.order = order;
  return launch(&m, stream);
}

}  // namespace rkmi
