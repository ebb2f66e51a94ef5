"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

Holds none of the method's arithmetic: only random draws and the workload recipes
(parameters of each benchmark configuration). NumPy only; callers move data to a device.
"""

import math

import numpy as np


def random_complex(n, seed=1234):
    """U[-1,1] + i U[-1,1], complex128."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)


# Workloads: the plane-wave impedance problem on the unit square, zero initial guess.
CFG_SMALL = dict(name="p1_k16_n64", k=16.0, n=64, p=1, s=1 + 0.5j, theta=math.pi / 7,
                 nu=2, omega=0.6, restart=50, tol=1e-8)
CFG_P1_LARGE = dict(name="p1_k400_n2048", k=400.0, n=2048, p=1, s=1 + 0.5j,
                    theta=math.pi / 7, nu=2, omega=0.6, restart=50, tol=1e-10)
CFG_SWEEP = dict(name="p2_k150_n512_sweep", k=150.0, n=512, p=2, nu=2, omega=0.6,
                 restart=50, tol=1e-8)
CFG_MIXED = dict(name="p3_k200_n256", k=200.0, n=256, p=3, s=1 + 0.5j, theta=math.pi / 7,
                 nu=2, omega=0.6, restart=50, tol=1e-10)


def sweep_betas(count=64, lo=0.05, hi=1.5):
    """beta_i evenly spaced in [lo, hi]."""
    return [lo + i * (hi - lo) / (count - 1) for i in range(count)]


def sweep_thetas(count=4, seed=0):
    """Incidence angles shared by every shift of the sweep."""
    return list(np.random.default_rng(seed).uniform(0.0, 2 * math.pi, count))


def serving_requests(count=2000, seed=1, rate=None, kmin=10.0, kmax=300.0, bmin=0.1, bmax=1.5,
                     khp_max=0.3, nmax=2048):
    """Request stream: per request draw (gap, log k, p, beta, theta) in that order.

    n = 2^m is the smallest power of two with k / (n p) <= khp_max, capped at nmax;
    gaps are exponential with mean 1/rate (all zero when rate is None).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        gap = rng.exponential(1.0 / rate) if rate else 0.0
        k = math.exp(rng.uniform(math.log(kmin), math.log(kmax)))
        p = int(rng.integers(1, 4))
        beta = rng.uniform(bmin, bmax)
        theta = rng.uniform(0.0, 2 * math.pi)
        n = 2
        while k / (n * p) > khp_max and n < nmax:
            n *= 2
        t += gap
        out.append(dict(id=i, t=t, k=k, p=p, n=n, beta=beta, theta=theta))
    return out


def shift_samples(count, seed=2, ells=(4, 5, 6, 7, 8, 9, 10), orders=(1, 2, 3)):
    """Samples of the shift search (Sec. 5, data generation): per sample draw the order p,
    then ell (h = 2^-ell), then k uniform in [3p / (16 h), 3p / (4 h)]; the right-hand side
    is drawn by sample_rhs from the sample's own seed."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        p = int(rng.choice(orders))
        ell = int(rng.choice(ells))
        h = 2.0 ** -ell
        k = float(rng.uniform(3 * p / (16 * h), 3 * p / (4 * h)))
        out.append(dict(id=i, p=p, ell=ell, h=h, n=2 ** ell, k=k, rhs_seed=seed * 100003 + i))
    return out


def sample_rhs(sample):
    """Right-hand side of a shift-search sample: every component uniform in [-1, 1], real
    (imaginary part zero), on the fine lattice of (p, h)."""
    M = sample["p"] * sample["n"] + 1
    rng = np.random.default_rng(sample["rhs_seed"])
    return rng.uniform(-1.0, 1.0, M * M) + 0j


def wedge_mu(n, levels=(0.45, 0.7, 1.0)):
    """Synthetic three-layer wedge profile mu in (0, 1], one value per cell of the n x n
    mesh (indexed [row j (y), column i (x)]), sampled at the cell centres: levels[0] below
    y = 0.2 + 0.3 x, levels[2] above y = 0.75 - 0.25 x, levels[1] in the wedge between
    (the two interfaces meet at x = 1)."""
    c = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(c, c, indexing="xy")
    mu = np.full((n, n), levels[1])
    mu[Y < 0.2 + 0.3 * X] = levels[0]
    mu[Y > 0.75 - 0.25 * X] = levels[2]
    return mu


def random_cells(n, lo, hi, seed):
    """Per-cell values uniform in [lo, hi] (n x n, indexed [row j, column i])."""
    return np.random.default_rng(seed).uniform(lo, hi, (n, n))


# Heterogeneous workload: the wedge profile with k_max = 400 on P1, h = 1/2048, the point
# source at (0.5, 0.55), g = 0.
CFG_WEDGE = dict(name="wedge_p1_kmax400_n2048", kmax=400.0, n=2048, p=1, source=(0.5, 0.55),
                 nu=2, omega=0.6, restart=50, tol=1e-8)
