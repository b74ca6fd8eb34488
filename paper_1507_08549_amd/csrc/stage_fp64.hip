// FP64 instantiation of the fused stage kernel.  Built with -ffp-contract=off:
// the only fused multiply-adds are the explicit ones, so every result is the
// same IEEE operation sequence as the CPU oracle's.
#include "stage_kernel.hpp"

namespace hy {
hipError_t launch_stage_fp64(const StageArgs& a, hipStream_t s) { return launch_stage<double>(a, s); }
}  // namespace hy
