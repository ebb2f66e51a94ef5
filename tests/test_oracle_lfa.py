"""Pins of the local Fourier analysis (Sec. 3) and parity of the vectorised calculator.

The oracle's symbols are checked against a brute-force twogrid operator on a periodic grid
(where the Fourier modes are exact eigenvectors, so the eigenvalues of the dense operator
are exactly those of the 4 x 4 symbols at the discrete low frequencies), against the
Galerkin identity of nested Q1 spaces and against the definition of the Jacobi smoother.
"""

import math

import numpy as np
import pytest

from oracle import lfa as O
from paper_2104_01439_amd import lfa as G


def _stencil_matrix(n, st):
    """Periodic n x n grid, 3 x 3 stencil st[b+1][a+1] (offsets a along x, b along y)."""
    N = n * n
    A = np.zeros((N, N), complex)
    for j in range(n):
        for i in range(n):
            for b in (-1, 0, 1):
                for a in (-1, 0, 1):
                    A[j * n + i, ((j + b) % n) * n + (i + a) % n] += st[b + 1][a + 1]
    return A


def _q1_stencil(lam, h):
    K = np.array([[-1, -1, -1], [-1, 8, -1], [-1, -1, -1]]) / 3
    M = np.array([[1, 4, 1], [4, 16, 4], [1, 4, 1]]) * h * h / 36
    return K - lam * M


def _prolongation(n):
    """Bilinear interpolation from the (n/2)^2 periodic coarse grid (fine point 2I + kappa
    receives w_kappa times the coarse value, w = [1 2 1]^T [1 2 1] / 4)."""
    nc = n // 2
    P = np.zeros((n * n, nc * nc))
    w = np.array([1, 2, 1]) / 2
    for J in range(nc):
        for I in range(nc):
            for b in (-1, 0, 1):
                for a in (-1, 0, 1):
                    P[((2 * J + b) % n) * n + (2 * I + a) % n, J * nc + I] += w[a + 1] * w[b + 1]
    return P


def _periodic_twogrid(n, k, h, sigma, omega, nu1, nu2):
    lam = k * k + 1j * k ** sigma
    L = _stencil_matrix(n, _q1_stencil(lam, h))
    L2 = _stencil_matrix(n // 2, _q1_stencil(lam, 2 * h))
    P = _prolongation(n)
    S = np.eye(n * n) - omega * np.diag(1 / np.diag(L)) @ L
    K = np.eye(n * n) - P @ np.linalg.solve(L2, P.T @ L)
    return (np.linalg.matrix_power(S, nu2) @ K @ np.linalg.matrix_power(S, nu1), L, L2, P)


@pytest.mark.parametrize("k,h,sigma,nu", [(8.0, 1 / 16, 1.5, 1), (20.0, 1 / 16, 1.0, 2),
                                          (4.0, 1 / 16, 2.0, 3)])
def test_symbols_equal_periodic_brute_force(k, h, sigma, nu):
    n = 16
    T, L, L2, P = _periodic_twogrid(n, k, h, sigma, 2 / 3, nu, nu)
    ev = np.linalg.eigvals(T)
    # discrete low frequencies 2 pi m / n, m in (-n/4, n/4]
    ms = range(-n // 4 + 1, n // 4 + 1)
    lev = []
    for m1 in ms:
        for m2 in ms:
            th = (2 * math.pi * m1 / n, 2 * math.pi * m2 / n)
            lev += list(np.linalg.eigvals(O.twogrid_matrix(th, k, h, sigma, 2 / 3, nu, nu)))
    lev = np.array(lev)
    assert len(lev) == len(ev) == n * n
    # every symbol eigenvalue is an eigenvalue of the operator, and the spectra agree
    d = np.abs(lev[:, None] - ev[None, :]).min(axis=1)
    assert d.max() <= 1e-9 * max(1.0, np.abs(ev).max())
    assert np.allclose(np.sort(np.abs(lev)), np.sort(np.abs(ev)), atol=1e-9)


def test_galerkin_coarse_operator_on_periodic_grid():
    """P^T L_h P = L_2h for nested Q1 spaces (the coarse stencil is the h -> 2h one)."""
    n = 16
    _, L, L2, P = _periodic_twogrid(n, 7.0, 1 / 16, 1.3, 2 / 3, 1, 1)
    assert np.abs(P.T @ L @ P - L2).max() <= 1e-13


def test_coarse_correction_is_a_projection():
    rng = np.random.default_rng(3)
    for _ in range(10):
        th = tuple(rng.uniform(-math.pi / 2, math.pi / 2, 2))
        K = O.twogrid_matrix(th, 30.0, 1 / 32, 1.4, 2 / 3, 0, 0)
        assert np.abs(K @ K - K).max() <= 1e-10


def test_smoother_symbol_is_jacobi_definition():
    rng = np.random.default_rng(4)
    k, h, s, w = 50.0, 1 / 64, 1.2, 0.6
    lam = k * k + 1j * k ** s
    for _ in range(10):
        th = tuple(rng.uniform(-math.pi, math.pi, 2))
        D = 8 / 3 - lam * h * h * 16 / 36          # centre of the Q1 stencil
        assert abs(O.symbol_S(th, lam, h, w) - (1 - w * O.symbol_Lh(th, lam, h) / D)) <= 1e-13


def test_rho_loc_shrinks_with_the_shift_and_sigma_c():
    # the example of Sec. 3: nu = 3, omega = 2/3, h = 2^-5, k h = 0.25
    h = 2.0 ** -5
    k = 0.25 / h
    rs = [O.rho_loc(k, h, s, n=48) for s in (1.0, 1.25, 1.5, 1.75, 2.0)]
    assert all(rs[i] >= rs[i + 1] - 1e-12 for i in range(4))
    sc = O.sigma_c(k, h, n=48, tol=1e-3)
    assert sc is not None and 1.0 <= sc <= 2.0
    if sc > 1.0:
        assert O.rho_loc(k, h, sc, n=48) < 1.0 <= O.rho_loc(k, h, sc - 2e-3, n=48)


@pytest.mark.parametrize("k,h,sigma", [(8.0, 1 / 32, 1.0), (100.0, 1 / 256, 1.5),
                                       (400.0, 1 / 1024, 1.8)])
def test_vectorised_calculator_equals_oracle(k, h, sigma):
    rng = np.random.default_rng(5)
    th = rng.uniform(-math.pi / 2, math.pi / 2, (6, 2))
    Tg = G.twogrid_symbols(th[:, 0], th[:, 1], k, h, sigma)
    for i in range(6):
        To = O.twogrid_matrix(tuple(th[i]), k, h, sigma)
        assert np.abs(Tg[i] - To).max() <= 1e-12 * max(1.0, np.abs(To).max())
    for axis in (True, False):
        assert abs(G.rho_loc(k, h, sigma, n=24, axis=axis) -
                   O.rho_loc(k, h, sigma, n=24, axis=axis)) <= 1e-12


def test_vectorised_sigma_c_equals_oracle():
    for kh, h in [(0.25, 2.0 ** -5), (0.5, 2.0 ** -6)]:
        k = kh / h
        assert G.sigma_c(k, h, n=32, tol=1e-3) == O.sigma_c(k, h, n=32, tol=1e-3)
