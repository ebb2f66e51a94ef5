"""Pins of the oracle's heterogeneous-k operator, Galerkin coarse operator and Gaussian
load vector (``oracle/hetero.py``) against textbook element matrices, closed-form
integrals, the constant-k special case and a dense solve."""

import math

import numpy as np
import pytest

from oracle.fem import Discretisation, prolongation
from oracle.hetero import (operator_cells, source_rhs, gaussian, TwoGridCells, ProblemCells)
from oracle.twogrid import TwoGrid
from paper_2104_01439_amd import inputs


def _rel(A, B):
    A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    B = B.toarray() if hasattr(B, "toarray") else np.asarray(B)
    return np.abs(A - B).max() / np.abs(B).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_constant_cells_equal_constant_operator(p):
    d = Discretisation(6, p)
    k, s = 7.5, 1 + 0.4j
    A = operator_cells(d, np.full((6, 6), k), np.full((6, 6), s))
    assert _rel(A, d.operator(k, s)) < 1e-14


def test_one_cell_mass_p1_textbook():
    """Raising s_c k_c^2 of one interior cell by delta adds -delta times the P1 mass of
    its two triangles, h^2/24 [2 1 1; 1 2 1; 1 1 2] each, at the cell's four vertices."""
    n, h = 5, 1 / 5
    d = Discretisation(n, 1)
    kc = inputs.random_cells(n, 2.0, 6.0, 3)
    sc = np.ones((n, n), complex)
    cx, cy, delta = 3, 1, 0.7
    k2 = kc.copy()
    k2[cy, cx] = math.sqrt(kc[cy, cx] ** 2 + delta)
    D = (operator_cells(d, k2, sc) - operator_cells(d, kc, sc)).toarray()
    M = d.M
    v00, v10, v11, v01 = (cy * M + cx, cy * M + cx + 1, (cy + 1) * M + cx + 1,
                          (cy + 1) * M + cx)
    E = np.zeros_like(D)
    u = h * h / 24
    for a, b, val in [(v00, v00, 4), (v11, v11, 4), (v10, v10, 2), (v01, v01, 2),
                      (v00, v11, 2), (v00, v10, 1), (v10, v11, 1), (v00, v01, 1),
                      (v01, v11, 1)]:
        E[a, b] += -delta * val * u
        if a != b:
            E[b, a] += -delta * val * u
    assert np.abs(D - E).max() < 1e-15


@pytest.mark.parametrize("p", [2, 3])
def test_one_cell_mass_total(p):
    """The same change for P2/P3 touches only the (p+1)^2 dofs of the cell and its entries
    sum to -delta h^2 (the basis sums to one, so sum_ij M_ij = area)."""
    n = 4
    d = Discretisation(n, p)
    kc = inputs.random_cells(n, 2.0, 6.0, 4)
    sc = 1 + 1j * inputs.random_cells(n, 0.1, 0.9, 5)
    cx, cy, delta = 1, 2, 1.3
    s2 = sc.copy()
    s2[cy, cx] += delta / kc[cy, cx] ** 2
    D = (operator_cells(d, kc, s2) - operator_cells(d, kc, sc)).toarray()
    M = d.M
    dofs = [(p * cy + j) * M + p * cx + i for j in range(p + 1) for i in range(p + 1)]
    mask = np.zeros(d.N, bool)
    mask[dofs] = True
    assert np.abs(D[~mask]).max() == 0 and np.abs(D[:, ~mask]).max() == 0
    assert abs(D.sum() - (-delta * d.h ** 2)) < 1e-14


def test_boundary_edge_k_p1():
    """Changing k of the corner cell (0, 0) with s k^2 held fixed changes only the
    impedance term -i k B on its bottom and left edges, h/6 [2 1; 1 2] each."""
    n, h = 4, 1 / 4
    d = Discretisation(n, 1)
    kc = np.full((n, n), 3.0)
    sc = np.full((n, n), 1 + 0.5j)
    k2, s2 = kc.copy(), sc.copy()
    k2[0, 0] = 5.0
    s2[0, 0] = sc[0, 0] * 9.0 / 25.0
    D = (operator_cells(d, k2, s2) - operator_cells(d, kc, sc)).toarray()
    M = d.M
    E = np.zeros_like(D)
    for (a, b) in [(0, 1), (0, M)]:           # bottom edge (0)-(1), left edge (0)-(M)
        for i, j, val in [(a, a, 2), (b, b, 2), (a, b, 1), (b, a, 1)]:
            E[i, j] += -1j * 2.0 * val * h / 6
    assert np.abs(D - E).max() < 1e-14


@pytest.mark.parametrize("side", ["bottom", "right", "top", "left"])
def test_boundary_edge_k_each_side_p1(side):
    """The same for one non-corner cell on each side: only the edge of that side, between
    the two boundary vertices of the cell, changes."""
    n, h = 5, 1 / 5
    d = Discretisation(n, 1)
    M = d.M
    cell = {"bottom": (2, 0), "right": (n - 1, 3), "top": (1, n - 1), "left": (0, 2)}[side]
    cx, cy = cell
    verts = {"bottom": (cy * M + cx, cy * M + cx + 1),
             "right": (cy * M + cx + 1, (cy + 1) * M + cx + 1),
             "top": ((cy + 1) * M + cx, (cy + 1) * M + cx + 1),
             "left": (cy * M + cx, (cy + 1) * M + cx)}[side]
    kc = inputs.random_cells(n, 2.0, 4.0, 8)
    sc = np.full((n, n), 1 + 0.3j)
    k2, s2 = kc.copy(), sc.copy()
    k2[cy, cx] = kc[cy, cx] + 1.5
    s2[cy, cx] = sc[cy, cx] * kc[cy, cx] ** 2 / k2[cy, cx] ** 2
    D = (operator_cells(d, k2, s2) - operator_cells(d, kc, sc)).toarray()
    E = np.zeros_like(D)
    a, b = verts
    for i, j, val in [(a, a, 2), (b, b, 2), (a, b, 1), (b, a, 1)]:
        E[i, j] += -1j * 1.5 * val * h / 6
    assert np.abs(D - E).max() < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3])
def test_galerkin_equals_coarse_cells(p):
    """With the coefficient constant on every coarse cell, P^T A P is the coarse operator
    assembled with the coarse-cell coefficients (nested spaces, exact integration)."""
    nc = 4
    kco = inputs.random_cells(nc, 3.0, 9.0, 11)
    sco = 1 + 1j * inputs.random_cells(nc, 0.05, 1.2, 12)
    kf = np.kron(kco, np.ones((2, 2)))
    sf = np.kron(sco, np.ones((2, 2)))
    fine, coarse = Discretisation(2 * nc, p), Discretisation(nc, p)
    P = prolongation(fine, coarse)
    G = P.T @ operator_cells(fine, kf, sf) @ P
    assert _rel(G, operator_cells(coarse, kco, sco)) < 1e-12


@pytest.mark.parametrize("p", [1, 2, 3])
def test_source_rhs_polynomial_is_mass_times_interpolant(p):
    """For f in the FE space the rule is exact: F = M f_I."""
    d = Discretisation(6, p)
    if p == 1:
        f = lambda x, y: 1.0 + 2.0 * x - 3.0 * y
    else:
        f = lambda x, y: 1.0 + 2.0 * x - 3.0 * y + 1.5 * x * y - 0.5 * y * y
    F = source_rhs(d, f)
    assert np.abs(F - d.Mass @ d.interpolate(f)).max() < 1e-15


def _g0(s, a):
    return 0.5 * math.sqrt(math.pi / a) * (math.erf(math.sqrt(a) * (1 - s)) + math.erf(math.sqrt(a) * s))


def _g1(s, a):
    return s * _g0(s, a) + (math.exp(-a * s * s) - math.exp(-a * (1 - s) ** 2)) / (2 * a)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_gaussian_source_moments(p):
    """sum_i F_i = int f and sum_i x_i F_i = int x f (the basis reproduces 1 and x) for
    f = 2 exp(-1000 |x - s|^2): closed forms with erf."""
    c = (0.5, 0.55)
    d = Discretisation(128 // p, p)
    F = source_rhs(d, gaussian(c))
    x, y = d.coords()
    a = 1000.0
    m0 = 2 * _g0(c[0], a) * _g0(c[1], a)
    mx = 2 * _g1(c[0], a) * _g0(c[1], a)
    my = 2 * _g0(c[0], a) * _g1(c[1], a)
    # the rule's error at this mesh is below 5e-14 (measured); 1e-12 leaves room
    assert abs(F.sum() - m0) / m0 < 1e-12
    assert abs((x * F).sum() - mx) / mx < 1e-12
    assert abs((y * F).sum() - my) / my < 1e-12
    assert np.abs(F.imag).max() == 0


@pytest.mark.parametrize("p", [1, 3])
def test_twogrid_cells_constant_equals_twogrid(p):
    n, k, s = 8, 9.0, 1 + 0.6j
    tgc = TwoGridCells(n, p, np.full((n, n), k), np.full((n, n), s), coarse_solver="dense")
    tg = TwoGrid(k, n, p, s, coarse_solver="dense")
    f = inputs.random_complex(tg.fine.N, seed=3)
    assert np.abs(tgc.vcycle(f) - tg.vcycle(f)).max() / np.abs(tg.vcycle(f)).max() < 1e-12


@pytest.mark.parametrize("p", [1, 2])
def test_problem_cells_solves_dense(p):
    """FGMRES with the heterogeneous twogrid cycle solves A_0 u = F (dense check)."""
    n = 12
    kc = 30.0 * inputs.wedge_mu(n)
    sc = 1 + 1j * kc ** -0.5                       # eps = k^{3/2} per cell
    pr = ProblemCells(n, p, kc, sc, coarse_solver="dense")
    F = pr.gaussian_rhs((0.5, 0.55))
    out = pr.solve(F, tol=1e-11)
    u = np.linalg.solve(pr.A0.toarray(), F)
    assert out["converged"]
    assert np.linalg.norm(out["u"] - u) / np.linalg.norm(u) < 1e-9
