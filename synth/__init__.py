"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This package only *generates inputs*: velocity models, the Ricker source
time function and the five workload geometries.  It holds none of the
solver's arithmetic (no stencil, no time stepping, no damping, no stability
analysis).  Both sides receive the same float32 arrays produced here; the
oracle promotes them to float64, the HIP path consumes them as they are.
"""
from .velocity import smooth_random, layered_perturbed, two_layer, smooth_along_z, request_layered, layered_profile
from .wavelet import ricker
from .workloads import Workload, workload, WORKLOADS, COURANT

__all__ = [
    "smooth_random", "layered_perturbed", "two_layer", "smooth_along_z", "request_layered", "layered_profile",
    "ricker", "Workload", "workload", "WORKLOADS", "COURANT",
]
