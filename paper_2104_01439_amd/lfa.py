"""Local Fourier analysis of the twogrid method for Q1 elements (Sec. 3), vectorised.

For the shifted local operator A(k, k^sigma) = K - (k^2 + i k^sigma) M on square Q1 elements
of side h (no boundary), damped Jacobi smoothing and an exact coarse solve on the 2h grid,
the twogrid error operator acts on the four harmonics of a low frequency theta as the 4 x 4
matrix T(theta) = S^nu2 (I - P L_2h^{-1} R L_h) S^nu1. rho_loc(sigma) is the largest
spectral radius over the low frequencies; sigma_c is the smallest exponent in [1, 2] with
rho_loc < 1, i.e. the twogrid method converges locally for sigma in [sigma_c, 2].

All frequencies of a grid are handled at once (numpy, batched 4 x 4 eigenvalues). Used on
the host to bound the sampling ranges of the shift search; it is not on the solve path.
"""

import numpy as np

_ALPHA = np.array([[0, 0], [1, 1], [1, 0], [0, 1]])


def _partner(t):
    return np.where(t < 0, t + np.pi, t - np.pi)


def twogrid_symbols(t1, t2, k, h, sigma, omega=2 / 3, nu1=3, nu2=3):
    """T(theta) for arrays of low frequencies (t1, t2): shape (..., 4, 4)."""
    t1 = np.asarray(t1, float)
    t2 = np.asarray(t2, float)
    lam = k * k + 1j * k ** sigma
    hh = h * h
    # the four harmonics of every frequency: (..., 4)
    T1 = np.stack([t1, _partner(t1), _partner(t1), t1], axis=-1)
    T2 = np.stack([t2, _partner(t2), t2, _partner(t2)], axis=-1)
    c1, c2 = np.cos(T1), np.cos(T2)
    Lh = (8 - 2 * c1 - 2 * c2 - 4 * c1 * c2) / 3 - lam * hh / 36 * (16 + 8 * c1 + 8 * c2 + 4 * c1 * c2)
    d = 8 / 3 - lam * hh * 16 / 36
    S = 1 - omega * Lh / d
    C1, C2 = np.cos(2 * t1), np.cos(2 * t2)
    L2 = (8 - 2 * C1 - 2 * C2 - 4 * C1 * C2) / 3 - lam * hh / 9 * (16 + 8 * C1 + 8 * C2 + 4 * C1 * C2)
    a1, a2 = np.cos(t1)[..., None], np.cos(t2)[..., None]
    P = np.concatenate([(1 + a1) * (1 + a2), (1 - a1) * (1 - a2), (1 - a1) * (1 + a2),
                        (1 + a1) * (1 - a2)], axis=-1)                   # (..., 4)
    # K = I - P (1/L2) (P^T / 4) diag(Lh)
    K = np.eye(4) - (P[..., :, None] * (0.25 * P * Lh)[..., None, :]) / L2[..., None, None]
    Sd1 = S ** nu1
    Sd2 = S ** nu2
    return Sd2[..., :, None] * K * Sd1[..., None, :]


def rho_loc(k, h, sigma, omega=2 / 3, nu1=3, nu2=3, n=64, axis=True):
    """Largest spectral radius over the low frequencies (-pi/2, pi/2]^2 on an n-point grid
    per axis (theta_2 = 0 only when axis is set), skipping theta = 0."""
    ts = -np.pi / 2 + np.pi * (np.arange(n) + 1) / n
    if axis:
        t1, t2 = ts, np.zeros_like(ts)
    else:
        t1, t2 = np.meshgrid(ts, ts, indexing="ij")
        t1, t2 = t1.ravel(), t2.ravel()
    keep = ~((t1 == 0) & (t2 == 0))
    T = twogrid_symbols(t1[keep], t2[keep], k, h, sigma, omega, nu1, nu2)
    return float(np.abs(np.linalg.eigvals(T)).max())


def sigma_c(k, h, omega=2 / 3, nu1=3, nu2=3, n=64, tol=1e-4):
    """Smallest sigma in [1, 2] with rho_loc(sigma) < 1 (bisection); 1.0 when sigma = 1
    converges already, None when sigma = 2 does not."""
    ok = lambda s: rho_loc(k, h, s, omega, nu1, nu2, n) < 1.0
    if ok(1.0):
        return 1.0
    if not ok(2.0):
        return None
    lo, hi = 1.0, 2.0
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if ok(mid):
            hi = mid
        else:
            lo = mid
    return hi
