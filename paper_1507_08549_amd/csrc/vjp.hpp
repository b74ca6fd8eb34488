// vjp.hpp -- launcher interface of the stage adjoint kernel.
#pragma once

#include "hydro_internal.hpp"

namespace hy {

// One Runge-Kutta stage W = U0 + b ((V - U0) + dt L(V)) transposed, with the
// LF speeds (ax, ay) held fixed:
//   out = b (lam + dt J_L(V)^T lam) + c0 add0 + c1 add1     (adjoint of V)
// (add0, add1 optional).  The adjoint of U0, (1 - b) lam, is not written:
// the caller adds the stages' shares where the step's adjoint is formed
// (through add0 / add1 of the first stage).  out may not alias lam, V, add0
// or add1.
struct VjpArgs {
  Geom g;
  double dt;
  int fp32;
  const double* V;
  const double* lam;
  double b;
  double ax, ay;
  double* out;
  const double* add0;
  double c0;
  const double* add1;
  double c1;
  double* ghost;  // scratch: adjoint of ghost cells, [2][3][ny][4] then [2][3][nx][4]
  size_t ghost_y_offset;  // offset (doubles) of the y part in ghost
  void* Gp;       // scratch: partial J_L^T lam between the x and y passes, 4 n values of the pass precision
};

hipError_t launch_stage_vjp(const VjpArgs& a, hipStream_t s);
hipError_t launch_stage_vjp_fp64(const VjpArgs& a, hipStream_t s);
hipError_t launch_stage_vjp_fp32(const VjpArgs& a, hipStream_t s);

}  // namespace hy
