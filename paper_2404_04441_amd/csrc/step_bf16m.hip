// Instantiation unit: the bfloat16 storage forward step kernels reading m as 16-bit codes.
#include "step_kernels.h"

namespace wave {

hipError_t launch_variant_bf16m(int v, const StepArgs &a, hipStream_t s) { return launch_variant<kBF16, false, true>(v, a, s); }

}  // namespace wave
