"""FP64 CPU oracle for the nodal DG Maxwell solver (test infrastructure only).

This package is a plain, slow, obviously-correct NumPy implementation of what
the GPU path computes: the nodal DG right-hand side for 2D TM and 3D Maxwell
on straight-sided simplices, the upwind numerical flux, the LIFT operator and
the five-stage low-storage RK4 time step.  It follows the paper's
"Construction of the Method" and "Implementation Aspects" sections
(eqs. claw, tm-maxwells, dg-weak, dg-strong, max2d-numflux,
dg-diff-local-to-global, dg-strong-matrix, dg-lift, dg-strong-explicit) and
the CPU right-hand side of the "Minimal Implementation" section.

It is TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with
the HIP library (``paper_1304_5546_amd``): the reference element, geometry,
connectivity, flux and time stepping are written here independently, in a
different language and, where the mathematics allows, by a different route
(coordinate matching for face neighbours, SciPy Jacobi polynomials for the
modal basis).

Every function is pinned in ``tests/test_oracle_*.py`` against closed forms,
invariants and brute force: polynomial exactness of differentiation, the
divergence theorem per element, closed-form PEC cavity modes, h-convergence of
order N+1, energy decay under the upwind flux (conservation under the central
flux), the stability polynomial of the RK scheme, the strong-form operator
against a weak form of eq. dg-weak assembled independently by quadrature
(``tests/test_oracle_weak_form.py``), and the energy and relative-L2
diagnostics against exact integrals of polynomial and piecewise-constant
fields (``tests/test_oracle_norms.py``).  Planted mistakes (a dropped 1/2,
a flipped sign, swapped material weights, a missing square root or
Jacobian) fail those pins.  Parity unpinned: none (the node-set parameter
alpha_opt and the CFL constant are shared *inputs*, not method arithmetic).
"""

from .element import RefElement2D, RefElement3D, lgl_nodes  # noqa: F401
from .mesh import Discretization2D, Discretization3D  # noqa: F401
from .maxwell import (  # noqa: F401
    LSRK4_A, LSRK4_B, LSRK4_C, Maxwell2D, Maxwell3D, cfl_dt, cavity_mode_2d,
    cavity_mode_3d,
)
