"""MI355X-native 8th-order acoustic wave-equation stencil (libwave).

The fused gfx950 step kernel, the checkpointed adjoint and the runtime live
in ``csrc/`` behind the C ABI of ``include/wave.h``; ``Solver`` and
``WaveFn`` are thin Python fronts over it.
"""
from ._lib import WaveError, WaveParams, LIB_PATH, EXPORTS  # noqa: F401


def __getattr__(name):
    # torch-dependent fronts are imported lazily so that the C-ABI checks work
    # without touching the GPU
    if name in ("Solver", "variant_count", "variant_info"):
        from . import solver
        return getattr(solver, name)
    if name == "WaveFn":
        from .autograd import WaveFn
        return WaveFn
    raise AttributeError(name)
