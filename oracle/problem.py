"""One Helmholtz solve as the paper sets it up (Sec. 4 and Sec. 5).

Test infrastructure (see the package header).

A_0 = A(k, 0) is the unshifted system matrix; the preconditioner is one twogrid
V(nu, nu)-cycle on A_eps with eps = beta k^2 (s = 1 + i beta); the outer method is
FGMRES(m) with a zero initial guess.
"""

import numpy as np

from .fem import Discretisation
from .twogrid import TwoGrid
from .fgmres import fgmres


class Problem:
    def __init__(self, k, n, p, s, nu=2, omega=0.6, coarse_solver="banded"):
        self.k, self.n, self.p, self.s = float(k), int(n), int(p), complex(s)
        self.tg = TwoGrid(self.k, self.n, self.p, self.s, nu, omega, coarse_solver)
        self.fine = self.tg.fine
        self.A0 = self.fine.operator(self.k, 1.0)

    @property
    def N(self):
        return self.fine.N

    def planewave_rhs(self, theta):
        return self.fine.planewave_rhs(self.k, theta)

    def apply_A0(self, x):
        return self.A0 @ x

    def solve(self, F, tol=1e-8, m=50, maxit=5000, record=False):
        return fgmres(self.apply_A0, self.tg.vcycle, F, tol=tol, m=m, maxit=maxit,
                      record=record)
