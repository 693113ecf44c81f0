"""FP64 CPU oracle for the 8th-order acoustic wave-equation stencil.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct reference the HIP path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it; the solver library never does, and it shares no code, tables or
constants with the library.  Inputs come from the separate ``synth``
package (float32 arrays, promoted to float64 here).

Arrays are indexed ``[z, y, x]`` (x fastest in memory); points are given as
``(ix, iy, iz)`` node triples.

What each module follows:

* ``coefficients`` -- the c_m of Eq. 1 (Sec. II), 8th order / radius 4
  (Sec. IV-A: R = 4), as exact rationals from Taylor moment conditions.
* ``operators`` -- the Laplacian of Eq. 1 with zero ghost nodes, the
  Cerjan sponge, the stability bound of the leapfrog scheme.
* ``forward`` -- the per-iteration wavefield update of Sec. II (leapfrog in
  time), with the sponge, point source and receivers.
* ``adjoint`` -- exact discrete adjoint of ``forward`` and the velocity
  gradient of the L2 waveform misfit.
* ``pointwise`` -- one step evaluated at chosen nodes (checks of grids too
  large for the full loop).
* ``energy``, ``analytic``, ``dense`` -- self-checks (discrete energy,
  constant-velocity Green's function, dense brute-force operator).
* ``storage`` -- 16-bit wavefield storage with power-of-two scaling
  (the paper is silent on precision; parity unpinned, see module header).
* ``cpml`` -- the CPML absorbing boundary (the paper's boundary, cited in
  Sec. II / IV-A without formulas; the formulation is a reading, see its
  header), pinned by textbook weights, the closed-form harmonic steady
  state of its memory recursion (update order), the continuous PML's
  reflection coefficient and memory kernel (profile and recursion
  coefficients), the undamped limit and absorption against a large-domain
  reference.
"""
from .coefficients import fd_coefficients, second_derivative_weights
from .operators import laplacian, sponge_profile, sponge_field, stability_courant, symbol_peak
from .forward import forward
from .adjoint import adjoint_fields, gradient, misfit
from .energy import discrete_energy
from .analytic import point_source_trace
from .dense import dense_laplacian
from .metrics import rel_l2, rel_max
from .pointwise import step_at
from . import storage
from . import cpml

__all__ = [
    "fd_coefficients", "second_derivative_weights", "laplacian", "sponge_profile", "sponge_field",
    "stability_courant", "symbol_peak", "forward", "adjoint_fields", "gradient", "misfit",
    "discrete_energy", "point_source_trace", "dense_laplacian", "rel_l2", "rel_max", "step_at",
]
