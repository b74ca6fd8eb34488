// vjp_launch.hpp -- launch sequence of one stage adjoint: x pass, y pass (2D;
// it also merges the x pass's ghost adjoints), then the fold of the remaining
// ghost adjoints (y in 2D, x in the 1D limit).
#pragma once

#include "vjp_kernel.hpp"

namespace hy {

template <typename R>
hipError_t launch_vjp_impl(const VjpArgs& a, hipStream_t s) {
  const Geom& g = a.g;
  double* gxb = a.ghost;
  double* gyb = a.ghost + a.ghost_y_offset;
  const int has_y = g.has_y;
  constexpr int NA = 58, NL = 4;  // cells per line and tile, lines per workgroup
  constexpr int NLY = sizeof(R) == 4 ? 16 : 8;  // columns per y-pass workgroup (16: 128-byte rows of the FP64 state)
  constexpr bool SY = true;
  {
    VjpPass p{a, a.Gp, has_y ? 0 : 1, gxb, nullptr};
    const int nb = ((g.nx + NA - 1) / NA) * ((g.ny + NL - 1) / NL);
    hipLaunchKernelGGL((vjp_line_kernel<R, 0, NL, false>), dim3(nb), dim3(64 * NL), 0, s, p);
  }
  if (has_y) {
    VjpPass p{a, a.Gp, 1, gyb, gxb};
    const int nb = ((g.ny + NA - 1) / NA) * ((g.nx + NLY - 1) / NLY);
    hipLaunchKernelGGL((vjp_line_kernel<R, 1, NLY, SY>), dim3(nb), dim3(64 * NLY), 0, s, p);
  }
  // (a periodic axis has no ghost adjoints to fold)
  const double scale = a.b * a.dt;
  if (!has_y && g.bc[0] != PERIODIC)  // in 2D the y pass has merged the x ghosts
    hipLaunchKernelGGL(vjp_fold_kernel<R>, dim3((4 * g.ny + 255) / 256), dim3(256), 0, s, g, 0,
                       (const double*)gxb, a.out, scale);
  else if (has_y && g.bc[2] != PERIODIC)
    hipLaunchKernelGGL(vjp_fold_kernel<R>, dim3((4 * g.nx + 255) / 256), dim3(256), 0, s, g, 1,
                       (const double*)gyb, a.out, scale);
  return hipGetLastError();
}

}  // namespace hy
