// FP64 instantiation of the stage adjoint.
#include "vjp_launch.hpp"

namespace hy {
hipError_t launch_stage_vjp_fp64(const VjpArgs& a, hipStream_t s) { return launch_vjp_impl<double>(a, s); }
hipError_t launch_stage_vjp(const VjpArgs& a, hipStream_t s) {
  return a.fp32 ? launch_stage_vjp_fp32(a, s) : launch_stage_vjp_fp64(a, s);
}
}  // namespace hy
