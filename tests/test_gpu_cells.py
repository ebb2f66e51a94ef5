"""GPU parity of the heterogeneous-k path (per-cell k and shift, Galerkin coarse operator,
Gaussian point source) through the C ABI against the oracle (``oracle/hetero.py``).

Tolerances as for constant k: 1e-12 relative for operator applies, transfers and the load
vector, 1e-10 for the coarse solve and the V-cycle, FGMRES iterations within +-1 and
solutions within 1e-8 at tolerance 1e-10; FP32 operators within 2e-6.
"""

import sys

import numpy as np
import pytest

from oracle.hetero import TwoGridCells, ProblemCells, operator_cells, source_rhs, gaussian
from paper_2104_01439_amd import inputs

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def hz(torch):
    from paper_2104_01439_amd import hz as h
    h.lib()
    return h


def cells(n, kmax, seed, kind):
    """k per cell (the wedge profile, or U[0.3, 1] k_max) and s = 1 + i k^{-1/2}
    (eps = k^{3/2} per cell)."""
    if kind == "wedge":
        kc = kmax * inputs.wedge_mu(n)
    else:
        kc = kmax * inputs.random_cells(n, 0.3, 1.0, seed)
    return kc, 1 + 1j * kc ** -0.5


# (n, p, kmax, kind): several coarse blocks, ragged lattice sizes, the smallest meshes
CASES = [(2, 1, 4.0, "random"), (40, 1, 25.0, "random"), (130, 1, 40.0, "wedge"),
         (2, 2, 5.0, "random"), (18, 2, 20.0, "random"), (4, 3, 6.0, "random"),
         (22, 3, 30.0, "wedge")]

_cache = {}


class _Case:
    def __init__(self, hz, torch, n, p, kmax, kind):
        _log(f"[cells] n={n} p={p} kmax={kmax} {kind}")
        self.torch = torch
        self.n, self.p = n, p
        self.kc, self.sc = cells(n, kmax, 100 + n + p, kind)
        self.gp = hz.Problem.cells(self.kc, self.sc, 1.0 / n, p, nu=2, omega=0.6)
        self.tg = TwoGridCells(n, p, self.kc, self.sc, nu=2, omega=0.6)
        self.A0 = operator_cells(self.tg.fine, self.kc, np.ones_like(self.sc))

    def dev(self, x):
        return self.torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda()

    def host(self, t):
        self.torch.cuda.synchronize()
        return t.cpu().numpy()


def case(hz, torch, c):
    if c not in _cache:
        for old in list(_cache):
            _cache.pop(old).gp.close()
        _cache[c] = _Case(hz, torch, *c)
    return _cache[c]


@pytest.mark.parametrize("c", CASES)
def test_cell_operators(hz, torch, c):
    t = case(hz, torch, c)
    tg = t.tg
    x = inputs.random_complex(tg.fine.N, seed=21)
    f = inputs.random_complex(tg.fine.N, seed=22)
    xc = inputs.random_complex(tg.coarse.N, seed=23)
    X, Fd, Xc = t.dev(x), t.dev(f), t.dev(xc)
    errs = {
        "A0": rel(t.host(t.gp.apply("A0", X)), t.A0 @ x),
        "AEPS": rel(t.host(t.gp.apply("AEPS", X)), tg.Aeps @ x),
        "JACOBI": rel(t.host(t.gp.apply("JACOBI", X, Fd)),
                      x + 0.6 * tg.dinv * (f - tg.Aeps @ x)),
        "COARSE_A": rel(t.host(t.gp.apply("COARSE_A", Xc)), tg.Ac @ xc),
        "RESID_RESTRICT": rel(t.host(t.gp.apply("RESID_RESTRICT", X, Fd)),
                              tg.P.T @ (f - tg.Aeps @ x)),
    }
    _log("  " + " ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    assert max(errs.values()) <= 1e-12


@pytest.mark.parametrize("c", CASES)
def test_cell_coarse_solve_and_vcycle(hz, torch, c):
    t = case(hz, torch, c)
    tg = t.tg
    r = inputs.random_complex(tg.coarse.N, seed=31)
    f = inputs.random_complex(tg.fine.N, seed=32)
    e_cs = rel(t.host(t.gp.apply("COARSE_SOLVE", t.dev(r))), tg.coarse_solve(r))
    e_vc = rel(t.host(t.gp.apply("VCYCLE", t.dev(f))), tg.vcycle(f))
    _log(f"  coarse solve {e_cs:.1e} vcycle {e_vc:.1e}")
    assert e_cs <= 1e-10 and e_vc <= 1e-10


@pytest.mark.parametrize("c", CASES)
def test_cell_operators_fp32(hz, torch, c):
    t = case(hz, torch, c)
    tg = t.tg
    x = inputs.random_complex(tg.fine.N, seed=41)
    e = rel(t.host(t.gp.apply("AEPS", t.dev(x), prec="mixed")), tg.Aeps @ x)
    _log(f"  AEPS fp32 {e:.1e}")
    assert e <= 2e-6


@pytest.mark.parametrize("p", [1, 2, 3])
def test_gaussian_rhs(hz, torch, p):
    n = 48 // p * 2
    pr = hz.Problem(10.0, 1.0 / n, p, 1 + 0.5j)
    F = pr.gaussian_rhs((0.5, 0.55)).cpu().numpy()
    Fo = source_rhs(pr_disc(n, p), gaussian((0.5, 0.55)))
    pr.close()
    e = rel(F, Fo)
    _log(f"  p={p} n={n}: load vector {e:.1e}")
    assert e <= 1e-12


def pr_disc(n, p):
    from oracle.fem import Discretisation
    return Discretisation(n, p)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n,p,kmax", [(64, 1, 60.0), (32, 2, 60.0), (24, 3, 60.0)])
def test_cell_solve_against_oracle(hz, torch, n, p, kmax, prec):
    """Wedge profile, point source at (0.5, 0.55), eps = k^{3/2} per cell, tol 1e-10."""
    kc, sc = cells(n, kmax, 0, "wedge")
    op = ProblemCells(n, p, kc, sc)
    Fo = op.gaussian_rhs((0.5, 0.55))
    ro = op.solve(Fo, tol=1e-10)
    pr = hz.Problem.cells(kc, sc, 1.0 / n, p, prec=prec)
    F = pr.gaussian_rhs((0.5, 0.55))
    u, r = pr.solve(F, tol=1e-10)
    pr.close()
    e = rel(u.cpu().numpy(), ro["u"])
    _log(f"  n={n} p={p} {prec}: iterations {r['iterations']} (oracle {ro['iterations']}), "
         f"u {e:.1e}, true residual {r['rel_res_true']:.1e}")
    assert r["converged"] == 1 and abs(r["iterations"] - ro["iterations"]) <= 1
    assert e <= 1e-8 and r["rel_res_true"] <= 1e-10


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cell_batched_equals_single(hz, torch, prec):
    """Two per-cell problems of one mesh in one batched call give bitwise their single
    solves; mixing a constant-k problem into the batch is refused."""
    n, p = 48, 2
    probs = []
    for seed in (1, 2):
        kc, sc = cells(n, 40.0, seed, "random")
        probs.append(hz.Problem.cells(kc, sc, 1.0 / n, p, prec=prec))
    Fs = [pr.gaussian_rhs((0.3 + 0.2 * i, 0.55)) for i, pr in enumerate(probs)]
    us, rs = hz.solve_batched(probs, Fs, 1, tol=1e-9)
    for i, pr in enumerate(probs):
        u1, r1 = pr.solve(Fs[i], tol=1e-9, history=False)
        assert r1["iterations"] == rs[i]["iterations"]
        assert torch.equal(u1, us[i])
    const = hz.Problem(40.0, 1.0 / n, p, 1 + 0.5j, prec=prec)
    with pytest.raises(hz.HZError) as ei:
        hz.solve_batched([probs[0], const], [Fs[0], Fs[0]], 1, tol=1e-9)
    assert ei.value.status == hz.HZ_EINVAL
    for pr in probs + [const]:
        pr.close()
    _log(f"  {prec}: iterations {[r['iterations'] for r in rs]}")


def test_release_cells():
    for key in list(_cache):
        _cache.pop(key).gp.close()


def test_cell_full_size(hz, torch):
    """The heterogeneous workload at full size: wedge, k_max = 400, P1, h = 1/2048 (4.2 M
    fine dofs). The coarse solve's residual through the (oracle-checked) Galerkin operator,
    and the FGMRES solve's true residual at tolerance 1e-8."""
    cfg = inputs.CFG_WEDGE
    n, p = cfg["n"], cfg["p"]
    kc, sc = cells(n, cfg["kmax"], 0, "wedge")
    _log(f"[cells] full size n={n} p={p} kmax={cfg['kmax']}")
    pr = hz.Problem.cells(kc, sc, 1.0 / n, p)
    r = torch.from_numpy(inputs.random_complex(pr.Nc, seed=7)).cuda()
    y = pr.apply("COARSE_SOLVE", r)
    Ay = pr.apply("COARSE_A", y)
    res = (torch.linalg.vector_norm(Ay - r) / torch.linalg.vector_norm(r)).item()
    F = pr.gaussian_rhs(cfg["source"])
    u, out = pr.solve(F, tol=cfg["tol"], history=False)
    pr.close()
    _log(f"  coarse residual {res:.1e}; solve {out['iterations']} iterations, "
         f"true residual {out['rel_res_true']:.1e}")
    assert res <= 1e-12
    assert out["converged"] == 1 and out["rel_res_true"] <= cfg["tol"]
