"""CPU FP64 oracle for the BBWADG acoustic right-hand side and LSRK4 step.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this package: only the
tests, the smoke check and the benchmark's CPU-baseline leg may use it.

The oracle is plain quadrature-based weight-adjusted DG (paper Section 3.1 and 3.3,
eq. (WADGform) and (pwadg)) in an orthonormal modal basis with dense matrices:

* polynomials of degree N on each affine tetrahedron, expanded in the orthonormal
  Dubiner (PKDO) basis, with mass, derivative and lift matrices formed by exact
  collapsed Gauss-Jacobi quadrature;
* neighbour traces evaluated at the same physical face points (no coefficient
  permutation maps);
* the weight-adjusted step dp/dt = P_q diag(c^2(x_q)) V_q r_p, where c^2 is either the
  per-element degree-M projection c^2_M (parity mode; then the Bernstein multiply +
  projection of the fast method computes the same thing exactly) or the true c^2;
* the 5-stage, 2N-storage fourth-order Runge-Kutta scheme of Carpenter and Kennedy.

It shares no code with the HIP path. Bernstein coefficients enter and leave only
through ``basis.py``, which evaluates the Bernstein basis from its definition
(paper Section 2).
"""
from .quadrature import gauss_jacobi, tet_rule, tri_rule  # noqa: F401
from .basis import dubiner_tet, bernstein_tet, bernstein_tri, multi_indices  # noqa: F401
from .mesh import Mesh  # noqa: F401
from .wadg import Oracle, LSRK4_A, LSRK4_B, LSRK4_C  # noqa: F401
