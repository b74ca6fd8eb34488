// FP32-bulk instantiation of the stage adjoint (FP64 accumulation of the
// stage combination).
#include "vjp_launch.hpp"

namespace hy {
hipError_t launch_stage_vjp_fp32(const VjpArgs& a, hipStream_t s) { return launch_vjp_impl<float>(a, s); }
}  // namespace hy
