"""Writes the stored expected values of the full-size parity tests, from the oracle only.

    python tests/golden/make_goldens.py [coarse] [coarse_b005] [solve] [solve_p1]

Each file holds results of the CPU FP64 oracle (``oracle/``) on seeded inputs
(``paper_2104_01439_amd/inputs.py``): sampled entries of the result at seeded indices, its
norm, and its inner products with seeded random vectors (global checks that see every
entry). The GPU tests recompute the same quantities from the library's results.

* ``coarse_p3_k200_n256.npz``: the direct coarse solve of the twogrid cycle (Sec. 4,
  Algorithm 1, coarsest level) for P3, k = 200, fine h = 1/256 (coarse h = 1/128,
  148 225 coarse dofs, lexicographic half-bandwidth 1158), shift s = 1 + 0.5i, right-hand
  side U[-1,1] + iU[-1,1] from seed 7; pivoted banded LU (LAPACK zgbtrf/zgbtrs).
* ``coarse_p2_k150_n512_b005.npz``: the same for P2, k = 150, fine h = 1/512 (coarse
  h = 1/256, 263 169 coarse dofs, half-bandwidth 1028) at the smallest shift of the shift
  sweep, s = 1 + 0.05i, where the unpivoted block elimination on the GPU sees the least
  damping.
* ``solve_p3_k200_n256.npz``: FGMRES(50) on A_0 (Sec. 4) with that twogrid preconditioner,
  plane-wave impedance data at theta = pi/7, tolerance 1e-10, zero initial guess:
  iteration count, residual history, true residual and the solution.
* ``solve_p1_k200_n1024.npz``: the same solve for P1, k = 200, fine h = 1/1024 (k h = 0.195,
  as for P1 at k = 400, h = 1/2048; 1 050 625 fine dofs, 263 169 coarse dofs,
  half-bandwidth 514).

Runs for about ten minutes and needs about 20 GB of memory.
"""

import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import Problem  # noqa: E402
from oracle.fem import Discretisation  # noqa: E402
from oracle.twogrid import BandedLU  # noqa: E402
from paper_2104_01439_amd import inputs  # noqa: E402

K, N_FINE, P, S, THETA = 200.0, 256, 3, 1 + 0.5j, math.pi / 7
NSAMPLE, NPROJ = 4096, 4


def sample_indices(n, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=min(NSAMPLE, n), replace=False))


def projections(x, seed0):
    """conj(v_i) . x for seeded U[-1,1] + iU[-1,1] vectors v_i."""
    return np.array([np.vdot(inputs.random_complex(x.size, seed=seed0 + i), x)
                     for i in range(NPROJ)])


def coarse(name="coarse_p3_k200_n256", k=K, n=N_FINE, p=P, s=S):
    t0 = time.time()
    disc = Discretisation(n // 2, p)
    Ac = disc.operator(k, s)
    lu = BandedLU(Ac)
    print(f"{name}: N_c={disc.N} factored in {time.time() - t0:.0f} s", flush=True)
    r = inputs.random_complex(disc.N, seed=7)
    y = lu.solve(r)
    res = np.linalg.norm(Ac @ y - r) / np.linalg.norm(r)
    idx = sample_indices(disc.N, 2024)
    np.savez(os.path.join(HERE, name + ".npz"), k=k, n=n, p=p, s=s, rhs_seed=7,
             idx=idx, y_idx=y[idx], y_norm=np.linalg.norm(y), proj=projections(y, 500),
             proj_seed=500, residual=res)
    print(f"{name}: residual {res:.2e}, |y| {np.linalg.norm(y):.6e} ({time.time() - t0:.0f} s)",
          flush=True)


def solve(name="solve_p3_k200_n256", k=K, n=N_FINE, p=P, s=S):
    t0 = time.time()
    pr = Problem(k, n, p, s, nu=2, omega=0.6)
    print(f"solve: N={pr.N} set up in {time.time() - t0:.0f} s", flush=True)
    F = pr.planewave_rhs(THETA)
    out = pr.solve(F, tol=1e-10, m=50)
    u = out["u"]
    true_res = np.linalg.norm(F - pr.A0 @ u) / np.linalg.norm(F)
    idx = sample_indices(pr.N, 2025)
    np.savez(os.path.join(HERE, name + ".npz"), k=k, n=n, p=p, s=s,
             theta=THETA, tol=1e-10, restart=50, iterations=out["iterations"],
             converged=out["converged"], hist=np.array(out["hist"]), rel_res_true=true_res,
             idx=idx, u_idx=u[idx], u_norm=np.linalg.norm(u), proj=projections(u, 600),
             proj_seed=600)
    print(f"solve: {out['iterations']} iterations, true residual {true_res:.2e} "
          f"({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    what = sys.argv[1:] or ["coarse", "coarse_b005", "solve", "solve_p1"]
    if "coarse" in what:
        coarse()
    if "coarse_b005" in what:
        coarse("coarse_p2_k150_n512_b005", 150.0, 512, 2, 1 + 0.05j)
    if "solve" in what:
        solve()
    if "solve_p1" in what:
        solve("solve_p1_k200_n1024", 200.0, 1024, 1, 1 + 0.5j)
