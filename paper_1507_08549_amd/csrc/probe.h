/*
 * probe.h -- measurement aid, built as its own library (libhydro_probe.so),
 * outside the solver's ABI (include/hydro.h).  The benchmark loads it to put
 * the kernels' roofline fractions beside what a plain FP64 fma stream reaches
 * on the same device.
 */
#ifndef HYDRO_PROBE_H
#define HYDRO_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Achievable FP64 vector fma rate of the current HIP device: eight independent
 * fma chains per work item, 8 workgroups of 256 work items per compute unit,
 * iters rounds (an fma counts 2 flops), one warm-up launch then one launch
 * timed with events on stream (a hipStream_t, NULL for the null stream).
 * *flops_per_s receives the rate.  Synchronises.  Returns 0, -1 for iters < 1
 * or a NULL output, -3 when a HIP call fails. */
int hydro_probe_fma_rate(int32_t iters, void* stream, double* flops_per_s);

#ifdef __cplusplus
}
#endif

#endif /* HYDRO_PROBE_H */
