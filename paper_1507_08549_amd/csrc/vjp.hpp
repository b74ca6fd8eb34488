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
  double* ghost;  // scratch for the adjoint of ghost cells
};

hipError_t launch_stage_vjp(const VjpArgs& a, hipStream_t s);

}  // namespace hy
