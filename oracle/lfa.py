"""Local Fourier analysis of the twogrid method for the Q1 discretisation (Sec. 3).

Test infrastructure (see the package header): plain loops over the frequencies, one 4 x 4
matrix at a time, following the symbols of Sec. 3 in the paper's order.

Setting (Sec. 3): no boundary, square Q1 elements of side h, the shifted local operator
A(k, eps) = K - (k^2 + i eps) M with eps = k^sigma, damped Jacobi smoothing (omega,
nu1 pre- and nu2 post-sweeps), bilinear prolongation, restriction and the coarse operator
on the 2h grid (the same stencil with 2h), exact coarse solve. For a low frequency theta
the four harmonics theta^(0,0), theta^(1,1), theta^(1,0), theta^(0,1) span an invariant
space on which the twogrid error operator acts as a 4 x 4 matrix
    T(theta) = S^nu2 (I - P L_2h^{-1} R L_h) S^nu1.

Readings where the text is garbled:
* the printed smoother stencil has corner entries that disagree with the printed symbol;
  the symbol (1 - omega L_h / D) is used;
* the printed prolongation symbols carry a factor 4 that belongs to the restriction (the
  FE restriction is the transpose of the interpolation); only the product P R enters;
* "k = 0.25 h" in the example is read as k h = 0.25;
* sigma_c is the smallest sigma in [1, 2] with rho_loc(sigma) < 1, the convergent set
  being [sigma_c, 2].
"""

import math

import numpy as np

HARMONICS = ((0, 0), (1, 1), (1, 0), (0, 1))


def bar(t):
    """The partner frequency of one component (shifted by pi into the other half)."""
    return t + math.pi if t < 0 else t - math.pi


def harmonic(theta, alpha):
    t1, t2 = theta
    return (bar(t1) if alpha[0] else t1, bar(t2) if alpha[1] else t2)


def symbol_Lh(theta, lam, h):
    c1, c2 = math.cos(theta[0]), math.cos(theta[1])
    return ((8 - 2 * c1 - 2 * c2 - 4 * c1 * c2) / 3
            - lam * h * h / 36 * (16 + 8 * c1 + 8 * c2 + 4 * c1 * c2))


def symbol_L2h(theta, lam, h):
    c1, c2 = math.cos(2 * theta[0]), math.cos(2 * theta[1])
    return ((8 - 2 * c1 - 2 * c2 - 4 * c1 * c2) / 3
            - lam * h * h / 9 * (16 + 8 * c1 + 8 * c2 + 4 * c1 * c2))


def symbol_S(theta, lam, h, omega):
    c1, c2 = math.cos(theta[0]), math.cos(theta[1])
    d = 8 / 3 - lam * h * h * 16 / 36
    return ((1 - omega) + omega * (2 / 3 + lam * h * h * 8 / 36) / d * c1
            + omega * (2 / 3 + lam * h * h * 8 / 36) / d * c2
            + omega * (4 / 3 + lam * h * h * 4 / 36) / d * c1 * c2)


def symbol_P(theta):
    """Column of the prolongation over the four harmonics (with the printed factor)."""
    c1, c2 = math.cos(theta[0]), math.cos(theta[1])
    return [(1 + c1) * (1 + c2), (1 - c1) * (1 - c2), (1 - c1) * (1 + c2), (1 + c1) * (1 - c2)]


def twogrid_matrix(theta, k, h, sigma, omega=2 / 3, nu1=3, nu2=3):
    """The 4 x 4 matrix T(theta, sigma) of the twogrid error operator."""
    lam = k * k + 1j * k ** sigma
    Lh = np.diag([symbol_Lh(harmonic(theta, a), lam, h) for a in HARMONICS])
    S = np.diag([symbol_S(harmonic(theta, a), lam, h, omega) for a in HARMONICS])
    P = np.array(symbol_P(theta), dtype=complex).reshape(4, 1)
    R = 0.25 * P.T
    L2 = symbol_L2h(theta, lam, h)
    K = np.eye(4) - P @ (R @ Lh) / L2
    return np.linalg.matrix_power(S, nu2) @ K @ np.linalg.matrix_power(S, nu1)


def spectral_radius(T):
    return max(abs(e) for e in np.linalg.eigvals(T))


def rho_loc(k, h, sigma, omega=2 / 3, nu1=3, nu2=3, n=64, axis=True):
    """sup of the spectral radius over the low frequencies (-pi/2, pi/2]^2 sampled on an
    n-point grid per axis; on the axis theta_2 = 0 only when axis is set (Sec. 3 restricts
    the search there after observing the maxima on the axes). theta = 0 is skipped (the
    constant mode)."""
    ts = [-math.pi / 2 + math.pi * (i + 1) / n for i in range(n)]
    best = 0.0
    for t1 in ts:
        for t2 in ([0.0] if axis else ts):
            if t1 == 0.0 and t2 == 0.0:
                continue
            best = max(best, spectral_radius(twogrid_matrix((t1, t2), k, h, sigma, omega, nu1,
                                                            nu2)))
    return best


def sigma_c(k, h, omega=2 / 3, nu1=3, nu2=3, n=64, tol=1e-4):
    """Smallest sigma in [1, 2] with rho_loc(sigma) < 1 (bisection; rho_loc decreases in
    sigma). Returns 1.0 if sigma = 1 converges, None if sigma = 2 does not."""
    f = lambda s: rho_loc(k, h, s, omega, nu1, nu2, n) < 1.0
    if f(1.0):
        return 1.0
    if not f(2.0):
        return None
    lo, hi = 1.0, 2.0
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if f(mid):
            hi = mid
        else:
            lo = mid
    return hi
