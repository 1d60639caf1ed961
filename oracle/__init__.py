"""CPU oracle of the CDI + GNBC time step -- TEST INFRASTRUCTURE.

A plain, slow, FP64 NumPy/SciPy implementation written from the paper
(Brown, Mirjalili, Khanwale, Mani, arXiv:2412.16843): the conservative
diffuse-interface phase-field flux with its sharpening term, no-flux walls,
one-sided wall stencils and linear extrapolation to the wall, the GNBC slip
(Models 1A..4B), the consistent momentum and energy-based surface-tension
stencils, RK4 with a projection at every stage, an exact pressure solve and
the diagnostics; cdi3d carries the same discretisation to three dimensions
(x and z periodic), with the slip as a wall-plane vector and the in-plane
curvature kappa_p of the curvature correction.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import it.  It shares no code with the HIP product path; both take their
inputs from the `workloads` module, which holds no arithmetic of the method.

Parity status: every function here is pinned by CPU tests against closed
forms, invariants, brute force or library routines (tests/test_oracle_*.py),
except the coupled dynamic contact-angle / steady Couette shape, whose only
published reference (molecular-dynamics data) is not available -- that
comparison is "parity unpinned" beyond the invariants it must satisfy.
"""
from . import cdi, cdi3d, poisson  # noqa: F401
