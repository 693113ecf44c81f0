// Instantiation unit: the float32 forward step kernels (2.5D shapes with and without the fused CPML x part and the cached policy, the semi-stencil, gmem and smem).
#include "step_kernels.h"

namespace wave {

hipError_t launch_variant_f32(int v, const StepArgs &a, hipStream_t s) { return launch_variant<kF32, false>(v, a, s); }
int blocks_variant_f32(int v, bool cpml) { return blocks_variant<kF32, false>(v, cpml); }

}  // namespace wave
