// Instantiation unit: the bfloat16 storage forward step kernels.
#include "step_kernels.h"

namespace wave {

hipError_t launch_variant_bf16(int v, const StepArgs &a, hipStream_t s) { return launch_variant<kBF16, false>(v, a, s); }
int blocks_variant_bf16(int v) { return blocks_variant<kBF16, false>(v, false); }

}  // namespace wave
