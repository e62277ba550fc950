// rk_batch.hpp -- ragged batches that mix networks of different sizes.
//
// A batch holds the systems of up to kMaxBatchNets compiled networks, each
// network's systems in their own struct-of-arrays block.  One persistent
// launch integrates all of them: every wave takes networks in a given order
// and runs the queue-refilled loop of persistent_loop over each network's
// queue until it is exhausted (a wave holds one network's code at a time, so
// lanes of a wave never diverge across networks); lanes freed by finished
// systems are refilled from the same queue, which compacts the live systems
// of a wave.  Operator-splitting substeps [t0 + k dt, t0 + (k + 1) dt] are
// restarts (Sec. 3): each substep is one queue reset and one launch, and a
// sequence of substeps can be captured in one HIP graph.
//
// Two plain forms serve as baselines: one launch over interleaved slots, each
// lane switching to its system's network, and one plain launch per network.
#pragma once

#include <cmath>
#include <cstring>
#include <vector>

#include "rk_group.hpp"
#include "rk_launch.hpp"

namespace rkmi {

constexpr int kMaxBatchNets = 4;
// queue heads kQueueStride 64-bit words apart (one 256-byte line each)
constexpr int kQueueStride = 32;

struct BatchNet {
  const double* prm;   // the network's uniform data
  int64_t n;           // its systems
  double* y;           // [N][n], integrated in place
  const double* g;     // [2][n]
  int32_t* status;     // [n] or null
  int32_t* stats;      // [kNStats][n] or null
  double* carry;       // [kCarryRows + N][n] or null
};

struct BatchParams {
  BatchNet net[kMaxBatchNets];
  int32_t order[kMaxBatchNets];    // network indices in the order waves take them
  int32_t refill[kMaxBatchNets];   // refill threshold per network
  int32_t map_net[kMaxBatchNets];  // interleaved form: network of slot-map code k
  int32_t n_net;
  unsigned long long* queues;      // [n_net * kQueueStride], heads zero at launch
  double* cols;                    // column workspace, col_block doubles per workgroup
  int64_t col_block;
};

// LDS doubles of a workgroup running Prob's persistent loop (one lane per
// system, or the group variant).
template <class Prob>
constexpr int persistent_lds_doubles() {
  if constexpr (Prob::kGroupLanes > 1)
    return group_lds_doubles<Prob>();
  else
    return kernel_lds_doubles<Prob, kMethodRkc>() * kLdsStride;
}

template <class... P>
constexpr int batch_lds_doubles() {
  int m = kLdsStride;
  ((m = persistent_lds_doubles<typename FastVariant<P>::type>() > m
            ? persistent_lds_doubles<typename FastVariant<P>::type>()
            : m),
   ...);
  ((m = kernel_lds_doubles<P, kMethodRkc>() * kLdsStride > m
            ? kernel_lds_doubles<P, kMethodRkc>() * kLdsStride
            : m),
   ...);
  return m;
}

template <class Prob>
constexpr int64_t col_block_of() {
  return (Prob::kGroupLanes == 1 && Prob::kColumns)
             ? (int64_t)slot_doubles<Prob, kMethodRkc>() * kLdsStride
             : 0;
}

// Column doubles one workgroup needs: the largest column-held network's block
// among the kernels' variants (Fast = the persistent kernel's, else the plain
// forms').
template <bool Fast, class... P>
constexpr int64_t batch_col_block() {
  int64_t m = 0;
  if constexpr (Fast)
    ((m = col_block_of<typename FastVariant<P>::type>() > m
              ? col_block_of<typename FastVariant<P>::type>()
              : m),
     ...);
  else
    ((m = col_block_of<P>() > m ? col_block_of<P>() : m), ...);
  return m;
}

template <class Prob>
__device__ void batch_run_net(const BatchNet& d, Ctl c, int refill, unsigned long long* queue,
                              double* lds, double* colbase) {
  c.refill = refill;
  if constexpr (Prob::kGroupLanes > 1) {
    group_persistent_loop<Prob, kMethodRkc>(d.prm, d.n, d.y, d.y, d.g, c, d.status, d.stats,
                                            queue, lds, nullptr, d.carry);
  } else {
    double* slot = Prob::kColumns ? colbase + threadIdx.x : lds + threadIdx.x;
    persistent_loop<Prob, kMethodRkc>(d.prm, d.n, d.y, d.y, d.g, c, d.status, d.stats, queue,
                                      slot, nullptr, d.carry);
  }
}

// The ragged kernel holds every network's code, so the register allocator
// sizes it for the largest (the 53-species group RKC) and would run one wave
// per SIMD; two waves, with a few hundred bytes of spills outside the stage
// loops, hide the group exchanges' LDS latency (1.8x on the four-network batch).
constexpr int kRaggedWavesPerEu = 2;

template <class... P>
__global__ __launch_bounds__(kLdsStride)
__attribute__((amdgpu_waves_per_eu(kRaggedWavesPerEu))) void ragged_kernel(BatchParams bp, Ctl c) {
  __shared__ __attribute__((aligned(16))) double lds[batch_lds_doubles<P...>()];
  double* const colbase = bp.cols ? bp.cols + (int64_t)blockIdx.x * bp.col_block : nullptr;
  for (int r = 0; r < bp.n_net; ++r) {
    const int k = bp.order[r];
    int idx = 0;
    ((idx++ == k ? batch_run_net<typename FastVariant<P>::type>(
                       bp.net[k], c, bp.refill[k], bp.queues + k * kQueueStride, lds, colbase)
                 : void()),
     ...);
  }
}

template <int = 0>
__global__ void batch_queue_reset(unsigned long long* queues, int n_net) {
  if ((int)threadIdx.x < n_net) queues[threadIdx.x * kQueueStride] = 0ull;
}

// Plain interleaved form: global slot i holds system (slot_map[i] & 0x0fffffff)
// of network slot_map[i] >> 28; each lane runs its own network's code.
template <class Prob>
__device__ void batch_plain_one(const BatchNet& d, const Ctl& c, int64_t local, double* slot) {
  integrate_system<Prob, kMethodRkc>(d.prm, d.n, local, d.y, d.y, d.g, c, d.status, d.stats,
                                     slot, d.carry);
}

template <class... P>
__global__ __launch_bounds__(kLdsStride) void interleaved_kernel(BatchParams bp, Ctl c,
                                                                 const int32_t* __restrict__ map,
                                                                 int64_t n_total) {
  __shared__ __attribute__((aligned(16))) double lds[batch_lds_doubles<P...>()];
  const int64_t i = (int64_t)blockIdx.x * kLdsStride + threadIdx.x;
  if (i >= n_total) return;
  const int32_t code = map[i];
  const int k = bp.map_net[(code >> 28) & (kMaxBatchNets - 1)];
  const int64_t local = code & 0x0fffffff;
  double* const colbase = bp.cols ? bp.cols + (int64_t)blockIdx.x * bp.col_block : nullptr;
  int idx = 0;
  ((idx++ == k ? batch_plain_one<P>(bp.net[k], c, local,
                                    P::kColumns ? colbase + threadIdx.x : lds + threadIdx.x)
               : void()),
   ...);
}

// Workgroups of the persistent ragged grid on the current device: waves_per_cu
// per compute unit (0: as many as the occupancy allows).
template <class... P>
int ragged_grid(int waves_per_cu, int64_t* grid) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ragged_kernel<P...>, kLdsStride, 0) !=
          hipSuccess)
    return kLaunchHip;
  if (per_cu < 1) per_cu = 1;
  if (waves_per_cu > 0 && waves_per_cu < per_cu) per_cu = waves_per_cu;
  *grid = (int64_t)cus * per_cu;
  return kLaunchOk;
}

// ---------------------------------------------------------------- host side

// Sets the launch-uniform bounds of the interval [t0, t1].
inline void ctl_interval(Ctl& c, double t0, double t1) {
  c.t0 = t0;
  c.t1 = t1;
  c.hmax = std::fabs(t1 - t0);
  c.hmin_rkc = 10.0 * kUround * std::fmax(std::fabs(t0), c.hmax);
}

// Bounds of substep s: [t0 + s dt, t0 + (s + 1) dt].
inline void substep_interval(const BatchArgs* a, int s, Ctl& c) {
  ctl_interval(c, a->t0 + (double)s * a->dt, a->t0 + (double)(s + 1) * a->dt);
}

constexpr size_t kBatchQueueBytes = (size_t)kBatchMaxNets * kQueueStride * sizeof(unsigned long long);

// A batch handle's captured graph of substeps and the arguments it was made for.
struct BatchGraphCache {
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<unsigned char> key;
};

inline void batch_free_cache(void* p) {
  BatchGraphCache* c = static_cast<BatchGraphCache*>(p);
  if (!c) return;
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->capture) (void)hipStreamDestroy(c->capture);
  delete c;
}

template <class... P>
BatchParams batch_params(const BatchArgs* a) {
  BatchParams bp{};
  for (int k = 0; k < kMaxBatchNets; ++k) {
    bp.net[k] = BatchNet{a->net[k].prm, a->net[k].n, a->net[k].y, a->net[k].g, a->net[k].status,
                         a->net[k].stats, a->net[k].carry};
    bp.order[k] = a->order[k];
    bp.map_net[k] = a->map_net[k];
    bp.refill[k] = a->refill[k] > 0 ? (a->refill[k] > kLdsStride ? kLdsStride : a->refill[k])
                                    : kDefaultRefill;
  }
  bp.n_net = (int32_t)sizeof...(P);
  unsigned char* ws = static_cast<unsigned char*>(a->ws);
  bp.queues = reinterpret_cast<unsigned long long*>(ws);
  bp.col_block = a->mode == kBatchPersistent ? batch_col_block<true, P...>()
                                             : batch_col_block<false, P...>();
  bp.cols = bp.col_block ? reinterpret_cast<double*>(ws + kBatchQueueBytes) : nullptr;
  return bp;
}

template <class... P>
int64_t batch_workspace(const BatchArgs* a) {
  if (a->mode == kBatchPersistent) {
    constexpr int64_t cb = batch_col_block<true, P...>() * (int64_t)sizeof(double);
    int64_t grid = 0;
    if (ragged_grid<P...>(a->waves_per_cu, &grid) != kLaunchOk) return -1;
    return (int64_t)kBatchQueueBytes + grid * cb;
  }
  constexpr int64_t cb = batch_col_block<false, P...>() * (int64_t)sizeof(double);
  if (a->mode == kBatchInterleaved)
    return (int64_t)kBatchQueueBytes + (a->n_total + kLdsStride - 1) / kLdsStride * cb;
  int64_t m = 0, k = 0;
  ((m = workspace_bytes<P, kMethodRkc>(kSchedPlain, a->net[k].n) > m
            ? workspace_bytes<P, kMethodRkc>(kSchedPlain, a->net[k].n)
            : m,
    ++k),
   ...);
  return m;
}

// Enqueues every substep of a ragged batch on the stream.
template <class... P>
int batch_enqueue(const BatchArgs* a, hipStream_t s) {
  if (a->mode == kBatchPerNet) {
    for (int st = 0; st < a->n_substeps; ++st) {
      int k = 0, rc = kLaunchOk;
      auto one = [&](auto tag) {
        using Prob = decltype(tag);
        LaunchArgs la{};
        la.method = kMethodRkc;
        la.schedule = kSchedPlain;
        la.n = a->net[k].n;
        la.y0 = a->net[k].y;
        la.y1 = a->net[k].y;
        la.g = a->net[k].g;
        la.prm = a->net[k].prm;
        la.ctl = a->ctl;
        substep_interval(a, st, la.ctl);
        la.status = a->net[k].status;
        la.stats = a->net[k].stats;
        la.carry = a->net[k].carry;
        la.ws = a->ws;
        la.ws_bytes = a->ws_bytes;
        if (rc == kLaunchOk && la.n > 0) rc = launch_method<Prob, kMethodRkc, false>(&la, s);
        ++k;
      };
      (one(P{}), ...);
      if (rc != kLaunchOk) return rc;
    }
    return kLaunchOk;
  }
  const BatchParams bp = batch_params<P...>(a);
  if (a->mode == kBatchInterleaved) {
    const int64_t blocks = (a->n_total + kLdsStride - 1) / kLdsStride;
    if (blocks <= 0) return kLaunchOk;
    if (blocks > 0x7fffffffLL) return kLaunchInvalid;
    for (int st = 0; st < a->n_substeps; ++st) {
      Ctl c = a->ctl;
      substep_interval(a, st, c);
      interleaved_kernel<P...><<<dim3((unsigned)blocks), dim3(kLdsStride), 0, s>>>(bp, c, a->map,
                                                                               a->n_total);
      if (hipGetLastError() != hipSuccess) return kLaunchHip;
    }
    return kLaunchOk;
  }
  int64_t grid = 0;
  if (ragged_grid<P...>(a->waves_per_cu, &grid) != kLaunchOk) return kLaunchHip;
  if (bp.col_block) {
    const int64_t fit = (int64_t)((a->ws_bytes - kBatchQueueBytes) /
                                  ((size_t)bp.col_block * sizeof(double)));
    if (grid > fit) grid = fit;
  }
  if (grid < 1) return kLaunchWorkspace;
  for (int st = 0; st < a->n_substeps; ++st) {
    Ctl c = a->ctl;
    substep_interval(a, st, c);
    batch_queue_reset<><<<1, kLdsStride, 0, s>>>(bp.queues, bp.n_net);
    ragged_kernel<P...><<<dim3((unsigned)grid), dim3(kLdsStride), 0, s>>>(bp, c);
    if (hipGetLastError() != hipSuccess) return kLaunchHip;
  }
  return kLaunchOk;
}

template <class... P>
int batch_launch(const BatchArgs* a, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t need = batch_workspace<P...>(a);
  if (need < 0) return kLaunchHip;
  if ((need > 0 && !a->ws) || a->ws_bytes < (size_t)need) return kLaunchWorkspace;
  if (!a->use_graph || a->n_substeps <= 0) return batch_enqueue<P...>(a, s);
  // the substeps captured once into a graph, replayed while the arguments match
  BatchGraphCache* cache = static_cast<BatchGraphCache*>(a->graph_cache);
  if (!cache) return kLaunchInvalid;
  BatchArgs keyed = *a;
  keyed.graph_cache = nullptr;
  std::vector<unsigned char> key(sizeof(BatchArgs));
  std::memcpy(key.data(), &keyed, sizeof(BatchArgs));
  if (!cache->exec || cache->key != key) {
    if (cache->exec) (void)hipGraphExecDestroy(cache->exec);
    if (cache->graph) (void)hipGraphDestroy(cache->graph);
    cache->exec = nullptr;
    cache->graph = nullptr;
    if (!cache->capture && hipStreamCreateWithFlags(&cache->capture, hipStreamNonBlocking) !=
                               hipSuccess)
      return kLaunchHip;
    if (hipStreamBeginCapture(cache->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return kLaunchHip;
    const int rc = batch_enqueue<P...>(a, cache->capture);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cache->capture, &g);
    if (rc != kLaunchOk || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc != kLaunchOk ? rc : kLaunchHip;
    }
    cache->graph = g;
    if (hipGraphInstantiate(&cache->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      cache->exec = nullptr;
      return kLaunchHip;
    }
    cache->key = key;
  }
  return hipGraphLaunch(cache->exec, s) == hipSuccess ? kLaunchOk : kLaunchHip;
}

}  // namespace rkmi
