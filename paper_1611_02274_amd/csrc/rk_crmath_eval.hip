// rk_crmath_eval.hip -- evaluates the kernels' exp / log / pow
// over arrays, on the host (the same source compiled for the CPU) or on the
// device, so that tests can check them.  fn: 0 exp(x), 1 log(x), 2 pow(x, y),
// 3 and 4: x^RN(1/3) and x^RN(2/3) from the RKC controllers' pair, 5: x^RN(1/3)
// alone, 6: x^-0.25, 7: x^-RN(0.2) as the RKCK controllers form them (y unused
// for 3 to 7).
// Not part of the public ABI.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "crmath.hpp"

namespace {

__host__ __device__ inline double eval_one(int fn, double x, double y) {
  switch (fn) {
    case 0: return rkmi::crm::cr_exp(x);
    case 1: return rkmi::crm::cr_log(x);
    case 3:
    case 4: {
      double p1 = 0.0, p2 = 0.0;
      rkmi::crm::pow_third_pair(x, p1, p2);
      return fn == 3 ? p1 : p2;
    }
    case 5: return rkmi::crm::pow_third_one(x);
    case 6: return rkmi::crm::pow_minus_quarter(x);
    case 7: return rkmi::crm::pow_minus_fifth(x);
    default: return rkmi::crm::cr_pow(x, y);
  }
}

__global__ void crmath_kernel(int fn, int64_t n, const double* __restrict__ x,
                              const double* __restrict__ y, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = eval_one(fn, x[i], y[i]);
}

}  // namespace

extern "C" int rkmi_crmath_host(int fn, int64_t n, const double* x, const double* y, double* out) {
  if (fn < 0 || fn > 7 || n < 0 || (n && (!x || !y || !out))) return -1;
  for (int64_t i = 0; i < n; ++i) out[i] = eval_one(fn, x[i], y[i]);
  return 0;
}

// x, y, out: device arrays of n doubles.
extern "C" int rkmi_crmath_device(int fn, int64_t n, const double* x, const double* y,
                                  double* out, void* stream) {
  if (fn < 0 || fn > 7 || n < 0 || (n && (!x || !y || !out))) return -1;
  if (n == 0) return 0;
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffffLL) return -1;
  crmath_kernel<<<dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream)>>>(
      fn, n, x, y, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
