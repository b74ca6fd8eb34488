// probe.hip -- achievable FP64 vector FMA rate of the device: a reference
// point for the roofline fractions the kernels report (a published peak is not
// always reachable by a plain instruction stream).  Built as libhydro_probe.so,
// separate from the solver library.
#include <hip/hip_runtime.h>

#include "probe.h"

namespace {

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

}  // namespace

extern "C" int hydro_probe_fma_rate(int32_t iters, void* stream, double* flops_per_s) {
  if (iters < 1 || !flops_per_s) return -1;
  hipStream_t st = (hipStream_t)stream;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -3;
  const int blocks = 8 * (cus > 0 ? cus : 1);  // 8 workgroups of 4 waves per compute unit
  double* sink = nullptr;
  if (hipMalloc(&sink, sizeof(double)) != hipSuccess) return -3;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 0;
  float ms = 0.0f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = -3;
  } else {
    hipLaunchKernelGGL(fma_probe_kernel, dim3(blocks), dim3(256), 0, st, sink, iters, 0.999999, 1e-7);
    if (hipGetLastError() != hipSuccess || hipEventRecord(e0, st) != hipSuccess) rc = -3;
    if (!rc) {
      hipLaunchKernelGGL(fma_probe_kernel, dim3(blocks), dim3(256), 0, st, sink, iters, 0.999999, 1e-7);
      if (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
          hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
          !(ms > 0.0f))
        rc = -3;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  if (rc) return rc;
  *flops_per_s = 2.0 * 8.0 * (double)iters * 256.0 * (double)blocks / (1e-3 * (double)ms);
  return 0;
}
