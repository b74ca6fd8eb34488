// FP32-bulk instantiation of the fused stage kernel (spatial operator in FP32,
// stage combination and reductions in FP64).  Built with contraction allowed.
#include "stage_kernel.hpp"

namespace hy {
hipError_t launch_stage_fp32(const StageArgs& a, hipStream_t s) { return launch_stage<float>(a, s); }
}  // namespace hy
