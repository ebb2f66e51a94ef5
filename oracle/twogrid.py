"""Twogrid V(nu, nu)-cycle on the shifted operator (Sec. 4, Algorithm 1, L = 2).

Test infrastructure (see the package header).

Called as the preconditioner with a zero initial guess:
    nu damped Jacobi sweeps  u <- u + omega D^{-1} (f - A_eps u),  D = diag(A_eps)
    restrict the residual    r_c = P^T (f - A_eps u)
    direct coarse solve      A_eps^{2h} e_c = r_c   (banded LU, factored once)
    prolong and correct      u <- u + P e_c
    nu damped Jacobi sweeps  (a diagonal smoother is its own transpose)
The coarse matrix is the rediscretisation of the shifted problem on the 2h mesh.
"""

import numpy as np
import scipy.sparse as sp
from scipy.linalg import lapack

from .fem import Discretisation, prolongation


class BandedLU:
    """Partially pivoted LU of a banded complex matrix (LAPACK zgbtrf / zgbtrs)."""

    def __init__(self, A):
        A = sp.coo_matrix(A)
        N = A.shape[0]
        bw = int(np.max(np.abs(A.row - A.col))) if A.nnz else 0
        kl = ku = bw
        ab = np.zeros((2 * kl + ku + 1, N), complex, order="F")
        ab[kl + ku + A.row - A.col, A.col] = A.data
        lu, piv, info = lapack.zgbtrf(ab, kl, ku, overwrite_ab=True)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrf info={info}")
        self.lu, self.piv, self.kl, self.ku, self.N = lu, piv, kl, ku, N

    def solve(self, b):
        x, info = lapack.zgbtrs(self.lu, self.kl, self.ku, np.asarray(b, complex), self.piv)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrs info={info}")
        return x


def jacobi_sweep(A, dinv, omega, u, f):
    """One damped Jacobi sweep u + omega D^{-1} (f - A u)."""
    return u + omega * dinv * (f - A @ u)


class TwoGrid:
    """Twogrid preconditioner for the P_p discretisation on n cells per side (n even)."""

    def __init__(self, k, n, p, s, nu=2, omega=0.6, coarse_solver="banded"):
        assert n % 2 == 0
        self.k, self.n, self.p, self.s = k, n, p, s
        self.nu, self.omega = nu, omega
        self.fine = Discretisation(n, p)
        self.coarse = Discretisation(n // 2, p)
        self.Aeps = self.fine.operator(k, s)
        self.dinv = 1.0 / self.Aeps.diagonal()
        self.P = prolongation(self.fine, self.coarse)
        self.Ac = self.coarse.operator(k, s)
        if coarse_solver == "banded":
            self.lu = BandedLU(self.Ac)
            self.coarse_solve = self.lu.solve
        else:                                   # dense brute force for tiny meshes
            Acd = self.Ac.toarray()
            self.coarse_solve = lambda r: np.linalg.solve(Acd, r)

    def smooth(self, u, f, sweeps):
        for _ in range(sweeps):
            u = jacobi_sweep(self.Aeps, self.dinv, self.omega, u, f)
        return u

    def restrict_residual(self, u, f):
        return self.P.T @ (f - self.Aeps @ u)

    def vcycle(self, f, u0=None):
        u = np.zeros_like(f, dtype=complex) if u0 is None else u0.astype(complex)
        u = self.smooth(u, f, self.nu)
        rc = self.restrict_residual(u, f)
        ec = self.coarse_solve(rc)
        u = u + self.P @ ec
        u = self.smooth(u, f, self.nu)
        return u
