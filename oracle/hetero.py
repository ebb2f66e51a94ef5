"""Heterogeneous wavenumber and the Gaussian point source (Sec. 6, the problem statement
that opens the numerical results: k(x) = k_max mu(x), f = 2 exp(-1000 |x - x_s|^2), g = 0).

Test infrastructure (see the package header).

Readings taken where the paper leaves the discrete form open:

* k is constant on every square cell of the fine mesh (both triangles of a cell share it),
  given as an n x n array indexed [cell row j (y), cell column i (x)]; a velocity image
  sampled per cell is of this form;
* the shift acts per cell: the mass term of cell c is weighted by s_c k_c^2 with a complex
  s_c = 1 + i beta_c (eps_c = beta_c k_c^2), the boundary term of an edge keeps the k of
  the cell it bounds (unshifted, as for constant k);
* the coarse operator of the twogrid cycle is the Galerkin product P^T A_eps P, which for
  nested spaces is the coarse form with the fine piecewise-constant coefficient integrated
  exactly (a coarse rediscretisation that samples k would differ from it);
* the load vector F_i = int f phi_i is integrated on every triangle with the collapsed
  Gauss-Legendre rule of q x q points (q = 6).
"""

import numpy as np
import scipy.sparse as sp

from .fem import Discretisation, prolongation, triangle_rule, ref_element
from .twogrid import BandedLU, jacobi_sweep
from .fgmres import fgmres


def _cell_values(disc, arr):
    """Per-element values of a per-cell array, in the element order of element_dofs."""
    n = disc.n
    a = np.asarray(arr)
    assert a.shape == (n, n)
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return a[cj.ravel(), ci.ravel()]


def operator_cells(disc, kcell, scell):
    """A = K - sum_c s_c k_c^2 M_c - i sum_{E on the boundary} k_E B_E (CSR, complex).

    M_c is the mass matrix of the two triangles of cell c, B_E the edge mass of boundary
    edge E and k_E the k of the cell that E bounds.
    """
    kcell = np.asarray(kcell, float)
    w = np.asarray(scell, complex) * kcell ** 2
    rows, cols, vals = [], [], []
    for kind in ("L", "U"):
        dofs = disc.element_dofs(kind)
        Ke = disc._em["K_" + kind]
        Me = disc._em["M_" + kind]
        nloc = Ke.shape[0]
        we = _cell_values(disc, w)
        rows.append(np.repeat(dofs, nloc, axis=1).ravel())
        cols.append(np.tile(dofs, (1, nloc)).ravel())
        vals.append((Ke.ravel()[None, :] - we[:, None] * Me.ravel()[None, :]).ravel())
    # boundary edges: bottom, right, top, left, edge i along the side
    n = disc.n
    i = np.arange(n)
    k_edge = np.concatenate([kcell[0, i], kcell[i, n - 1], kcell[n - 1, i], kcell[i, 0]])
    from .fem import edge_mass
    E = edge_mass(disc.p, disc.h)
    bd, _ = disc.boundary_edges()
    q = disc.p + 1
    rows.append(np.repeat(bd, q, axis=1).ravel())
    cols.append(np.tile(bd, (1, q)).ravel())
    vals.append((-1j * k_edge[:, None] * E.ravel()[None, :]).ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(disc.N, disc.N))
    return A.tocsr()


def source_rhs(disc, fun, q=6):
    """F_i = sum over triangles T of int_T fun phi_i, each by the q x q collapsed rule."""
    el = ref_element(disc.p)
    xi, eta, wt = triangle_rule(q)
    Phi = el.phi(xi, eta)                            # (nq, nloc)
    h = disc.h
    n = disc.n
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x0 = (ci.ravel() * h)[:, None]
    y0 = (cj.ravel() * h)[:, None]
    F = np.zeros(disc.N, complex)
    for kind in ("L", "U"):
        # T_L: x = v0 + h (xi + eta, eta); T_U: x = v0 + h (xi, xi + eta); |det J| = h^2
        if kind == "L":
            x = x0 + h * (xi + eta)[None, :]
            y = y0 + h * eta[None, :]
        else:
            x = x0 + h * xi[None, :]
            y = y0 + h * (xi + eta)[None, :]
        fv = fun(x, y)                               # (nel, nq)
        contrib = h * h * (fv * wt[None, :]) @ Phi   # (nel, nloc)
        np.add.at(F, disc.element_dofs(kind).ravel(), contrib.ravel())
    return F


def gaussian(center, amp=2.0, width=1000.0):
    """f(x) = amp exp(-width |x - center|^2)."""
    sx, sy = center
    return lambda x, y: amp * np.exp(-width * ((x - sx) ** 2 + (y - sy) ** 2))


class TwoGridCells:
    """Twogrid V(nu, nu)-cycle (Sec. 4, Algorithm 1) on the per-cell shifted operator with
    the Galerkin coarse operator."""

    def __init__(self, n, p, kcell, scell, nu=2, omega=0.6, coarse_solver="banded"):
        assert n % 2 == 0
        self.n, self.p, self.nu, self.omega = n, p, nu, omega
        self.fine = Discretisation(n, p)
        self.coarse = Discretisation(n // 2, p)
        self.Aeps = operator_cells(self.fine, kcell, scell)
        self.dinv = 1.0 / self.Aeps.diagonal()
        self.P = prolongation(self.fine, self.coarse)
        self.Ac = (self.P.T @ self.Aeps @ self.P).tocsr()
        if coarse_solver == "banded":
            self.lu = BandedLU(self.Ac)
            self.coarse_solve = self.lu.solve
        else:
            Acd = self.Ac.toarray()
            self.coarse_solve = lambda r: np.linalg.solve(Acd, r)

    def vcycle(self, f):
        u = np.zeros_like(f, dtype=complex)
        for _ in range(self.nu):
            u = jacobi_sweep(self.Aeps, self.dinv, self.omega, u, f)
        ec = self.coarse_solve(self.P.T @ (f - self.Aeps @ u))
        u = u + self.P @ ec
        for _ in range(self.nu):
            u = jacobi_sweep(self.Aeps, self.dinv, self.omega, u, f)
        return u


class ProblemCells:
    """FGMRES(m) on A_0 = A(k(x), 0) preconditioned by TwoGridCells on A_eps."""

    def __init__(self, n, p, kcell, scell, nu=2, omega=0.6, coarse_solver="banded"):
        self.n, self.p = int(n), int(p)
        self.kcell = np.asarray(kcell, float)
        self.scell = np.asarray(scell, complex)
        self.tg = TwoGridCells(self.n, self.p, self.kcell, self.scell, nu, omega,
                               coarse_solver)
        self.fine = self.tg.fine
        self.A0 = operator_cells(self.fine, self.kcell, np.ones_like(self.scell))

    @property
    def N(self):
        return self.fine.N

    def gaussian_rhs(self, center, q=6):
        return source_rhs(self.fine, gaussian(center), q)

    def solve(self, F, tol=1e-8, m=50, maxit=5000, record=False):
        return fgmres(lambda x: self.A0 @ x, self.tg.vcycle, F, tol=tol, m=m, maxit=maxit,
                      record=record)
