// probe.hip -- achievable FP64 vector FMA rate of the device: a reference
// point for the roofline fractions the kernels report (a published peak is not
// always reachable by a plain instruction stream).
#include <hip/hip_runtime.h>

#include "hydro_internal.hpp"

namespace hy {

// Eight independent fma chains per work item (enough to cover the FMA
// latency), `iters` rounds; the result is stored only if it matches an
// impossible value, so the chains cannot be removed.
__global__ __launch_bounds__(256) void fma_probe_kernel(double* out, int iters, double a, double b) {
  double x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = 1e-3 * (double)(threadIdx.x + k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = __builtin_fma(x[k], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  if (s == -12345.678) out[0] = s;
}

hipError_t launch_fma_probe(double* out, int iters, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(fma_probe_kernel, dim3(blocks), dim3(256), 0, s, out, iters, 0.999999, 1e-7);
  return hipGetLastError();
}

}  // namespace hy
