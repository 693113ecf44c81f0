// Instantiation unit: the IEEE-half storage forward step kernels reading m as 16-bit codes.
#include "step_kernels.h"

namespace wave {

hipError_t launch_variant_f16m(int v, const StepArgs &a, hipStream_t s) { return launch_variant<kF16, false, true>(v, a, s); }

}  // namespace wave
