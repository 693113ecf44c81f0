// Instantiation unit: the IEEE-half storage forward step kernels.
#include "step_kernels.h"

namespace wave {

hipError_t launch_variant_f16(int v, const StepArgs &a, hipStream_t s) { return launch_variant<kF16, false>(v, a, s); }
int blocks_variant_f16(int v) { return blocks_variant<kF16, false>(v, false); }

}  // namespace wave
