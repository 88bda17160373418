"""FP64 CPU oracle for the semi-implicit 1D-space electron BTE step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call or
link this package: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the GPU path; the only
module both consume is ``workloads`` (seeded inputs, no solver arithmetic).

The oracle is a plain, slow, direct transcription of the paper's discretization
("Hybrid fluid-BTE solver" section):

* ``basis``      Chebyshev-Gauss-Lobatto collocation in x, Gauss-Legendre
                 ordinates and spherical harmonics in polar angle, clamped cubic
                 B-splines in speed, composite Gauss quadrature.
* ``operators``  mass matrices, collision operator (eq. c_en_mat_1d) and its
                 gas-temperature correction (eq. c_T0_mat_1d), velocity-space
                 advection (eq. adv_v_ws), projections (eq. proj_ops), spatial
                 advection (eq. A_x) and moment vectors.
* ``step``       the semi-implicit step (eq. bte_semi_implicit): X(dt/2), field,
                 V(dt) by a dense LU solve per spatial point, X(dt/2); moments;
                 the transposed (adjoint) step and parameter gradients.

Every function cites the passage it follows.  Readings of passages that are
silent, garbled or ambiguous are documented in the repository design notes and
restated in the docstring where they are used.
"""
from .basis import (cgl_nodes, cheb_diff, gl_nodes, sph_harm_m0, sph_harm_m0_deriv,
                    bspline_knots, bspline_basis, bspline_basis_deriv)
from .operators import Operators, build_operators
from .semi_implicit import (x_half_step, x_half_step_T, v_step, field_half, step, moments,
                   initial_state, adjoint_step, run)

__all__ = [
    "cgl_nodes", "cheb_diff", "gl_nodes", "sph_harm_m0", "sph_harm_m0_deriv",
    "bspline_knots", "bspline_basis", "bspline_basis_deriv",
    "Operators", "build_operators",
    "x_half_step", "x_half_step_T", "v_step", "field_half", "step", "moments",
    "initial_state", "adjoint_step", "run",
]
