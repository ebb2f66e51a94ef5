"""CPU FP64 oracle for the twogrid-preconditioned FGMRES Helmholtz solve.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, links or runs this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use it. It shares no code with the HIP path.

What it computes (Drzisga, Koeppl, Wohlmuth, arXiv 2104.01439):

* the finite-element Helmholtz problem with an impedance boundary (Sec. 2, the
  boundary value problem and its sesquilinear form, the system matrix
  A(k, eps) = K - M(k, eps) - iB(k)), discretised here with P_p Lagrange
  elements (p = 1, 2, 3) on the uniform right-triangle mesh of the unit square;
* the twogrid V(nu, nu)-cycle on the shifted operator (Sec. 4, Algorithm 1) with a
  damped Jacobi smoother, the canonical FE prolongation, its transpose as
  restriction and an exact (banded LU) coarse solve;
* right-preconditioned flexible GMRES on the unshifted operator (Sec. 4, after
  Saad 1993), restarted every m steps, stopping on the relative residual.

Every function is written from the mathematics, in plain NumPy/SciPy, FP64 complex.
Pins for each part live in ``tests/test_oracle_*.py``.

Parity status: every function is pinned (closed forms, invariants, brute force, exact
solutions); the only unpinned quantities are iteration counts at full size, which the
paper does not print for this element and data.
"""

from .fem import Discretisation, ref_element, element_matrices
from .twogrid import BandedLU, TwoGrid
from .fgmres import fgmres
from .problem import Problem

__all__ = ["Discretisation", "ref_element", "element_matrices", "BandedLU",
           "TwoGrid", "fgmres", "Problem"]
