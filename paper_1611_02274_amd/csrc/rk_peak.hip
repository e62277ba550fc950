// rk_peak.hip -- FP64 vector-ALU throughput probe, the measured ceiling that the
// benchmark reports beside the chip's published FP64 vector peak.
// mode 0: sixteen independent chains of v_fma_f64 per lane (2 flops each);
// mode 1: sixteen independent chains alternating multiplies and adds (1 flop
// each), the instruction mix of kernels that keep a*b + c unfused.
// Not part of the public ABI.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kPeakBlocks = 256 * 16;
constexpr int kPeakThreads = 256;
constexpr int kChains = 16;

template <int Mode>
__global__ __launch_bounds__(kPeakThreads) void peak_kernel(int64_t iters, double b, double c,
                                                            double* __restrict__ out) {
  const int64_t tid = (int64_t)blockIdx.x * kPeakThreads + threadIdx.x;
  double a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = 1.0 + 1e-3 * (double)(k + (int)(tid & 7));
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
      if (Mode == 0)
        a[k] = __builtin_fma(a[k], b, c);
      else
        a[k] = (k & 1) ? a[k] + c : a[k] * b;
    }
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[tid] = s;
}

}  // namespace

// Threads one launch runs (the length of `out`).
extern "C" int64_t rkmi_peak_threads(void) { return (int64_t)kPeakBlocks * kPeakThreads; }

// Enqueues one launch of `iters` iterations on the stream; out: device array of
// rkmi_peak_threads() doubles.  *flops receives the launch's FP64 operation count.
extern "C" int rkmi_peak_fp64(int mode, int64_t iters, double* out, double* flops, void* stream) {
  if ((mode != 0 && mode != 1) || iters <= 0 || !out || !flops) return -1;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // b slightly below one and c tiny keep every chain finite and normal
  if (mode == 0)
    peak_kernel<0><<<dim3(kPeakBlocks), dim3(kPeakThreads), 0, s>>>(iters, 0.999999, 1e-9, out);
  else
    peak_kernel<1><<<dim3(kPeakBlocks), dim3(kPeakThreads), 0, s>>>(iters, 0.999999, 1e-9, out);
  *flops = (double)kPeakBlocks * kPeakThreads * (double)iters * kChains * (mode == 0 ? 2.0 : 1.0);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
