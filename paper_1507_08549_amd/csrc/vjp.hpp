// vjp.hpp -- launcher interface of the stage adjoint kernel.
#pragma once

#include "hydro_internal.hpp"

namespace hy {

// One Runge-Kutta stage W = U0 + b ((V - U0) + dt L(V)) transposed:
//   out  = b (lam + dt J_L(V)^T lam) + (acc ? acc : 0)     (adjoint of V)
//   side = (side_in ? side_in : 0) + (1 - b) lam            (adjoint of U0), if side
// with the LF speeds (ax, ay) held fixed.  out may alias acc, side may alias
// side_in; neither may alias lam or V.
struct VjpArgs {
  Geom g;
  double dt;
  int fp32;
  const double* V;
  const double* lam;
  double b;
  double ax, ay;
  double* out;
  const double* acc;
  double* side;
  const double* side_in;
  double* ghost;  // scratch: adjoint of ghost cells, [2][3][ny][4] then [2][3][nx][4]
  size_t ghost_y_offset;  // offset (doubles) of the y part in ghost
  double* Gp;     // scratch state: partial J_L^T lam between the x and y passes
};

hipError_t launch_stage_vjp(const VjpArgs& a, hipStream_t s);
hipError_t launch_stage_vjp_fp64(const VjpArgs& a, hipStream_t s);
hipError_t launch_stage_vjp_fp32(const VjpArgs& a, hipStream_t s);

}  // namespace hy
