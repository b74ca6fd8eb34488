// reduce.hip -- whole-grid reductions: the LF / CFL speeds of a state (when no
// producing stage has accumulated them) and the compensated conservation sums.
// Built with -ffp-contract=off (same primitive-variable arithmetic as the
// stage kernel).
#include "stage_kernel.hpp"

namespace hy {

__global__ void clear_slots_kernel(Ctl* ctl) {
  const int t = threadIdx.x;  // one sub-slot per work item
  if (t >= NSUB) return;
  for (int s = 0; s < 3; ++s)
    for (int k = 0; k < 3; ++k) ctl->slot[s][t][k] = 0ull;
}

hipError_t launch_clear_slots(Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(clear_slots_kernel, dim3(1), dim3(64), 0, s, ctl);
  return hipGetLastError();
}

// max over cells of |u|+c, |v|+c and c+(|u|+|v|): per-block maxima into
// partial[b][0..2] (partial[b][3] = 1 if rho <= 0, p <= 0 or c is not finite
// in the block), then one block merges them (no atomics).
constexpr int RED_THREADS = 256;
constexpr int RED_MAX_BLOCKS = 256;

__global__ __launch_bounds__(RED_THREADS) void alpha_partial_kernel(Geom g, const double* U,
                                                                    double* partial) {
  const size_t n = (size_t)g.nx * g.ny;
  double amax = 0.0, bmax = 0.0, smax = 0.0;
  bool bad = false;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    const double r = U[q], mx = U[n + q], my = U[2 * n + q], E = U[3 * n + q];
    const Prim<double> w = prim(r, mx, my, E, g.gamma, g.gm1);
    bad |= !(r > 0.0) || !(w.p > 0.0) || !__builtin_isfinite(w.c);
    amax = __builtin_fmax(amax, __builtin_fabs(w.u) + w.c);
    bmax = __builtin_fmax(bmax, __builtin_fabs(w.v) + w.c);
    smax = __builtin_fmax(smax, w.c + (__builtin_fabs(w.u) + __builtin_fabs(w.v)));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    amax = __builtin_fmax(amax, __shfl_xor(amax, off));
    bmax = __builtin_fmax(bmax, __shfl_xor(bmax, off));
    smax = __builtin_fmax(smax, __shfl_xor(smax, off));
  }
  __shared__ double red[RED_THREADS / 64][3];
  const int wave = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    red[wave][0] = amax;
    red[wave][1] = bmax;
    red[wave][2] = smax;
  }
  const int anybad = __syncthreads_or(bad ? 1 : 0);
  if (threadIdx.x == 0) {
    for (int k = 1; k < RED_THREADS / 64; ++k) {
      amax = __builtin_fmax(amax, red[k][0]);
      bmax = __builtin_fmax(bmax, red[k][1]);
      smax = __builtin_fmax(smax, red[k][2]);
    }
    partial[blockIdx.x * 4 + 0] = amax;
    partial[blockIdx.x * 4 + 1] = bmax;
    partial[blockIdx.x * 4 + 2] = smax;
    partial[blockIdx.x * 4 + 3] = anybad ? 1.0 : 0.0;
  }
}

// Merge the partial maxima into ring slot `slot` (sub-slot 0 holds the max,
// the other sub-slots zero) and clear the two other slots.  One wavefront.
__global__ void alpha_final_kernel(const double* partial, int nb, Ctl* ctl, int slot) {
  const int t = threadIdx.x;
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = t; b < nb; b += 64)
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = __builtin_fmax(m[k], partial[b * 4 + k]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = __builtin_fmax(m[k], __shfl_xor(m[k], off));
  if (t < NSUB) {
    for (int k = 0; k < 3; ++k) {
      ctl->slot[slot][t][k] = t == 0 ? as_bits(m[k]) : 0ull;
      ctl->slot[(slot + 1) % 3][t][k] = 0ull;
      ctl->slot[(slot + 2) % 3][t][k] = 0ull;
    }
  }
  if (t == 0 && m[3] != 0.0) atomicOr(&ctl->flag, 1);
}

int alpha_blocks(const Geom& g) {
  const size_t n = (size_t)g.nx * g.ny;
  size_t nb = (n + RED_THREADS * 8 - 1) / (RED_THREADS * 8);
  if (nb < 1) nb = 1;
  if (nb > RED_MAX_BLOCKS) nb = RED_MAX_BLOCKS;
  return (int)nb;
}

hipError_t launch_alpha_reduce(const Geom& g, const double* U, Ctl* ctl, int slot, double* partial,
                               hipStream_t s) {
  const int nb = alpha_blocks(g);
  hipLaunchKernelGGL(alpha_partial_kernel, dim3(nb), dim3(RED_THREADS), 0, s, g, U, partial);
  hipLaunchKernelGGL(alpha_final_kernel, dim3(1), dim3(64), 0, s, (const double*)partial, nb, ctl, slot);
  return hipGetLastError();
}

// --------------------------------------------------- compensated sums

// Neumaier's addition of b into the pair (s, c).
__device__ __forceinline__ void neu_add(double& s, double& c, double b) {
  const double t = s + b;
  if (__builtin_fabs(s) >= __builtin_fabs(b)) c += (s - t) + b;
  else c += (b - t) + s;
  s = t;
}

// Merge pair (s2, c2) into (s, c).
__device__ __forceinline__ void neu_merge(double& s, double& c, double s2, double c2) {
  neu_add(s, c, s2);
  c += c2;
}

constexpr int SUM_THREADS = 256;

int sums_blocks(const Geom& g) {
  const size_t n = (size_t)g.nx * g.ny;
  size_t nb = (n + SUM_THREADS * 16 - 1) / (SUM_THREADS * 16);
  if (nb < 1) nb = 1;
  if (nb > 1024) nb = 1024;
  return (int)nb;
}

// Fixed partition: block b owns a contiguous chunk; thread t walks it with
// stride SUM_THREADS; pairs are merged in a fixed tree.  Deterministic.
__global__ __launch_bounds__(SUM_THREADS) void sums_partial_kernel(Geom g, const double* U,
                                                                   double* partial) {
  const size_t n = (size_t)g.nx * g.ny;
  const size_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const size_t beg = (size_t)blockIdx.x * chunk;
  size_t end = beg + chunk;
  if (end > n) end = n;
  double s[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0};
  const double two_pi = 6.283185307179586;
  for (size_t q = beg + threadIdx.x; q < end; q += SUM_THREADS) {
    const int i = (int)(q % (size_t)g.nx);
    double vol = g.dx * g.dy;
    if (g.cyl) vol = (two_pi * (g.xlo + ((double)i + 0.5) * g.dx)) * vol;
#pragma unroll
    for (int k = 0; k < 4; ++k) neu_add(s[k], c[k], U[k * n + q] * vol);
  }
  __shared__ double ss[4][SUM_THREADS], sc[4][SUM_THREADS];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ss[k][threadIdx.x] = s[k];
    sc[k][threadIdx.x] = c[k];
  }
  __syncthreads();
  for (int stride = SUM_THREADS / 2; stride > 0; stride >>= 1) {
    if ((int)threadIdx.x < stride) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double a = ss[k][threadIdx.x], ac = sc[k][threadIdx.x];
        neu_merge(a, ac, ss[k][threadIdx.x + stride], sc[k][threadIdx.x + stride]);
        ss[k][threadIdx.x] = a;
        sc[k][threadIdx.x] = ac;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) {
    partial[blockIdx.x * 8 + threadIdx.x] = ss[threadIdx.x][0];
    partial[blockIdx.x * 8 + 4 + threadIdx.x] = sc[threadIdx.x][0];
  }
}

__global__ void sums_final_kernel(const double* partial, int nb, double* out) {
  const int k = threadIdx.x;
  if (k >= 4) return;
  double s = 0.0, c = 0.0;
  for (int b = 0; b < nb; ++b) neu_merge(s, c, partial[b * 8 + k], partial[b * 8 + 4 + k]);
  out[k] = s + c;
}

hipError_t launch_sums(const Geom& g, const double* U, double* partial, int nb, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(sums_partial_kernel, dim3(nb), dim3(SUM_THREADS), 0, s, g, U, partial);
  hipLaunchKernelGGL(sums_final_kernel, dim3(1), dim3(64), 0, s, partial, nb, out);
  return hipGetLastError();
}

}  // namespace hy
