"""Pins of the oracle's solver: exact solutions, brute force, Krylov identities.

Covers ``oracle/twogrid.py``, ``oracle/fgmres.py`` and ``oracle/problem.py``.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import Problem, fgmres
from oracle.fem import Discretisation, ref_element, triangle_rule, planewave
from oracle.twogrid import BandedLU, TwoGrid


def _fe_errors(d, uh, k, th):
    """L2 and H1-seminorm errors of uh against the plane wave, by element quadrature."""
    el = ref_element(d.p)
    xi, eta, wt = triangle_rule(8)
    Phi = el.phi(xi, eta)
    Gx, Gy = el.grad(xi, eta)
    c, s = np.cos(th), np.sin(th)
    h, n = d.h, d.n
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ci, cj = ci.ravel(), cj.ravel()
    e2 = e1 = 0.0
    for kind, J in (("L", np.array([[h, h], [0, h]])), ("U", np.array([[h, 0], [h, h]]))):
        U = uh[d.element_dofs(kind)]
        det = abs(np.linalg.det(J))
        G = np.linalg.inv(J).T
        X = ci[:, None] * h + J[0, 0] * xi[None, :] + J[0, 1] * eta[None, :]
        Y = cj[:, None] * h + J[1, 0] * xi[None, :] + J[1, 1] * eta[None, :]
        ue = np.exp(1j * k * (X * c + Y * s))
        uq = U @ Phi.T
        gxr, gyr = U @ Gx.T, U @ Gy.T
        gx = G[0, 0] * gxr + G[0, 1] * gyr
        gy = G[1, 0] * gxr + G[1, 1] * gyr
        e2 += det * np.sum(wt[None, :] * abs(uq - ue) ** 2)
        e1 += det * np.sum(wt[None, :] * (abs(gx - 1j * k * c * ue) ** 2 +
                                          abs(gy - 1j * k * s * ue) ** 2))
    return np.sqrt(e2), np.sqrt(e1)


@pytest.mark.parametrize("p,ns", [(1, [128, 256, 512]), (2, [32, 64, 128, 256]), (3, [16, 32, 64])])
def test_planewave_convergence_order(p, ns):
    """FE solution of the impedance problem converges to the exact plane wave at the
    optimal rates: p+1 in L2, p in the H1 seminorm."""
    k, th = 16.0, np.pi / 7
    errs = []
    for n in ns:
        d = Discretisation(n, p)
        u = spla.spsolve(d.operator(k).tocsc(), d.planewave_rhs(k, th))
        errs.append(_fe_errors(d, u, k, th))
    errs = np.array(errs)
    r2 = np.log2(errs[:-1, 0] / errs[1:, 0])
    r1 = np.log2(errs[:-1, 1] / errs[1:, 1])
    assert np.all(np.abs(r2[-2:] - (p + 1)) < 0.15), r2
    assert np.all(np.abs(r1[-2:] - p) < 0.15), r1


@pytest.mark.parametrize("p", [1, 2, 3])
def test_banded_lu_matches_dense(p):
    d = Discretisation(6, p)
    A = d.operator(8.0, 1 + 0.4j)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(d.N) + 1j * rng.standard_normal(d.N)
    x = BandedLU(A).solve(b)
    xd = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_twogrid_coarse_correction_is_projection(p):
    """nu = 0: for f = A_eps P x_c the V-cycle returns P x_c (Galerkin coarse operator)."""
    tg = TwoGrid(7.0, 8, p, 1 + 0.5j, nu=0)
    rng = np.random.default_rng(2)
    xc = rng.standard_normal(tg.coarse.N) + 1j * rng.standard_normal(tg.coarse.N)
    f = tg.Aeps @ (tg.P @ xc)
    z = tg.vcycle(f)
    assert np.linalg.norm(z - tg.P @ xc) <= 1e-11 * np.linalg.norm(tg.P @ xc)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_twogrid_is_linear_and_contracts_for_strong_shift(p):
    """The V-cycle is a linear map B; for beta = 1 and kh/p <= 0.3 the twogrid iteration
    on A_eps contracts: rho(I - B A_eps) < 1 (checks smoother and correction signs)."""
    k, n = 4.0, 4
    tg = TwoGrid(k, n, p, 1 + 1.0j, nu=2, omega=0.6, coarse_solver="dense")
    N = tg.fine.N
    Bm = np.stack([tg.vcycle(e) for e in np.eye(N, dtype=complex)], axis=1)
    rng = np.random.default_rng(0)
    f1 = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    f2 = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    assert np.linalg.norm(tg.vcycle(f1 + 2j * f2) - (Bm @ f1 + 2j * (Bm @ f2))) < 1e-10
    E = np.eye(N) - Bm @ tg.Aeps.toarray()
    rho = max(abs(np.linalg.eigvals(E)))
    assert rho < 1.0, rho
    # and the same iteration with a wrong-signed smoother correction diverges
    Ebad = np.eye(N) + np.diag(0.6 * tg.dinv) @ tg.Aeps.toarray()
    assert max(abs(np.linalg.eigvals(Ebad))) > 1.0


@pytest.mark.parametrize("p,n", [(1, 2), (1, 4), (1, 8), (2, 2), (2, 4), (3, 2), (3, 4)])
def test_fgmres_matches_dense_solve(p, n):
    k = 5.0
    pr = Problem(k, n, p, 1 + 0.5j, coarse_solver="dense")
    F = pr.planewave_rhs(0.9)
    ud = np.linalg.solve(pr.A0.toarray(), F)
    r = pr.solve(F, tol=1e-13, m=pr.N + 1)
    assert r["converged"]
    assert r["iterations"] <= pr.N
    assert np.linalg.norm(r["u"] - ud) <= 1e-10 * np.linalg.norm(ud)


def test_fgmres_arnoldi_relation_and_orthonormality():
    pr = Problem(12.0, 16, 2, 1 + 0.5j)
    F = pr.planewave_rhs(1.3)
    m = 12
    r = pr.solve(F, tol=1e-30, m=m, maxit=m, record=True)
    cols = [c[2] for c in r["cycles"] if c[0] == "col"]
    V, Z = [c for c in r["cycles"] if c[0] == "basis"][0][1:]
    Hbar = np.zeros((m + 1, m), complex)
    for j, col in enumerate(cols):
        Hbar[: j + 2, j] = col
    AZ = np.stack([pr.apply_A0(z) for z in Z], axis=1)
    assert np.linalg.norm(AZ - V.T @ Hbar) <= 1e-12 * np.linalg.norm(AZ)
    G = V.conj() @ V.T
    assert np.abs(G - np.eye(m + 1)).max() <= 1e-12


def test_fgmres_exact_preconditioner_one_iteration():
    pr = Problem(10.0, 8, 1, 1 + 0.5j)
    A = pr.A0.toarray()
    F = pr.planewave_rhs(0.4)
    r = fgmres(pr.apply_A0, lambda v: np.linalg.solve(A, v), F, tol=1e-10)
    assert r["iterations"] == 1 and r["converged"]


def test_fgmres_estimate_equals_true_residual_at_cycle_end():
    pr = Problem(20.0, 32, 1, 1 + 0.5j)
    F = pr.planewave_rhs(np.pi / 7)
    m = 10
    for its in (m, 2 * m, 3 * m):
        r = pr.solve(F, tol=1e-30, m=m, maxit=its)
        assert not r["converged"] and r["iterations"] == its
        est = r["hist"][-1]
        assert abs(est - r["true_rel_res"]) <= 1e-10 * r["true_rel_res"] + 1e-14


def test_fgmres_restarted_converges_to_fe_solution():
    pr = Problem(16.0, 64, 1, 1 + 0.5j)
    F = pr.planewave_rhs(np.pi / 7)
    ud = spla.spsolve(pr.A0.tocsc(), F)
    r = pr.solve(F, tol=1e-10, m=10)
    assert r["converged"] and r["true_rel_res"] <= 1e-10
    assert r["iterations"] > 10                       # at least one restart happened
    assert np.linalg.norm(r["u"] - ud) <= 1e-7 * np.linalg.norm(ud)
    assert np.all(np.diff(r["hist"][:10]) <= 1e-15)   # GMRES residual is monotone in a cycle
    assert 0 < r["rho"] < 1


def test_fgmres_edge_cases():
    pr = Problem(16.0, 8, 1, 1 + 0.5j)
    r = pr.solve(np.zeros(pr.N, complex))
    assert r["iterations"] == 0 and r["converged"] and np.all(r["u"] == 0)
    F = pr.planewave_rhs(0.3)
    r = pr.solve(F, tol=1e-30, maxit=3)
    assert r["iterations"] == 3 and not r["converged"]
