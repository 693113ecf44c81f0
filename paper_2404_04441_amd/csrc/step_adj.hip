// Instantiation unit: the float32 adjoint step kernels (two z queues, fused imaging).
#include "step_kernels.h"

namespace wave {

hipError_t launch_variant_adj(int v, const StepArgs &a, hipStream_t s) { return launch_variant<kF32, true>(v, a, s); }

}  // namespace wave
