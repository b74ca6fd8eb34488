// vjp_launch.hpp -- launch sequence of one stage adjoint: y pass (2D: the y
// part into a partial sum, and the y ghosts' adjoints), x pass (sources, the
// x part, the partial sum and the y ghosts merged, the stage combination),
// then the fold of the x ghosts' adjoints.
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
  if (has_y) {
    VjpPass p{a, a.Gp, 0, gyb, nullptr};
    const int nb = ((g.ny + NA - 1) / NA) * ((g.nx + NLY - 1) / NLY);
    hipLaunchKernelGGL((vjp_line_kernel<R, 1, NLY, true>), dim3(nb), dim3(64 * NLY), 0, s, p);
  }
  {
    VjpPass p{a, a.Gp, 1, gxb, has_y ? gyb : nullptr};
    const int nb = ((g.nx + NA - 1) / NA) * ((g.ny + NL - 1) / NL);
    hipLaunchKernelGGL((vjp_line_kernel<R, 0, NL, false>), dim3(nb), dim3(64 * NL), 0, s, p);
  }
  // the x ghosts (a periodic axis has none)
  if (g.bc[0] != PERIODIC)
    hipLaunchKernelGGL(vjp_fold_kernel<R>, dim3((4 * g.ny + 255) / 256), dim3(256), 0, s, g, 0,
                       (const double*)gxb, a.out, a.b * a.dt);
  return hipGetLastError();
}

}  // namespace hy
