"""Near-optimal shift exponent by golden-section search (Sec. 5, data generation).

Test infrastructure (see the package header).

For a sample (k, n = 1/h, p) and a right-hand side F (Sec. 5: components uniform in [-1, 1],
g = 0), the objective of a shift exponent sigma is the average reduction of the true
residual of an FGMRES solve preconditioned with the twogrid cycle on A(k, k^sigma):
    rho(sigma) = (r_end / r_0)^(1 / end),  r = ||A_0 u - F||,
with the solve stopped at relative residual 1e-8 or after 50 iterations, no restarts. The
exponent is located on [1, 2] by golden-section search (Kiefer 1953) to a bracket of 1e-2.
The shift eps = k^sigma enters as the multiplier s = 1 + i k^(sigma - 2) of the k^2 mass
term. In each step the bracket [a, b] with inner points c < d keeps [a, d] if
rho(c) < rho(d), else [c, b] (ties move the lower end).
"""

import math

from .problem import Problem

GOLDEN = (math.sqrt(5.0) - 1.0) / 2.0


def golden_section(f, lo, hi, tol):
    """Minimises a unimodal f on [lo, hi]; returns (midpoint of the final bracket, list of
    (x, f(x)) in evaluation order)."""
    a, b = lo, hi
    c = b - GOLDEN * (b - a)
    d = a + GOLDEN * (b - a)
    fc, fd = f(c), f(d)
    trace = [(c, fc), (d, fd)]
    while b - a > tol:
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - GOLDEN * (b - a)
            fc = f(c)
            trace.append((c, fc))
        else:
            a, c, fc = c, d, fd
            d = a + GOLDEN * (b - a)
            fd = f(d)
            trace.append((d, fd))
    return 0.5 * (a + b), trace


def shift_multiplier(k, sigma):
    """s with eps = k^sigma = Im(s) k^2 and Re(s) = 1."""
    return 1.0 + 1j * k ** (sigma - 2.0)


def objective(k, n, p, sigma, F, tol=1e-8, maxit=50, nu=2, omega=0.6):
    """rho(sigma) of one solve (0 when F = 0 needs no iteration)."""
    pr = Problem(k, n, p, shift_multiplier(k, sigma), nu=nu, omega=omega)
    out = pr.solve(F, tol=tol, m=maxit, maxit=maxit)
    if out["iterations"] == 0:
        return 0.0
    return out["true_rel_res"] ** (1.0 / out["iterations"])


def search(k, n, p, F, lo=1.0, hi=2.0, tol=1e-2, solve_tol=1e-8, maxit=50, nu=2, omega=0.6):
    return golden_section(lambda s: objective(k, n, p, s, F, solve_tol, maxit, nu, omega),
                          lo, hi, tol)
