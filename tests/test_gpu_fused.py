"""The fused V-cycle passes against their two-pass forms: the first post-smoothing sweep with
the coarse-grid correction staged in the stencil tile (Alg. 1: add coarse grid correction,
then postsmoothing; P1, P2) and the residual with the restriction in one pass (Alg. 1:
restrict residual; P1), against the same computation with the correction as its own
prolongation-add pass and the residual written then restricted (HZ_FUSE_PC=0, HZ_FUSE_RR=0,
read once per process, so that side runs in a child process). V-cycles, the residual
restriction and whole FGMRES solves are bitwise equal in FP64 and with FP32 operators, for
nu = 1, 2, 3, ragged tiles, a batched solve, P1-P3, and the orders and operators that keep
the two-pass forms (P3, per-point operators). Both sides are also checked against the
oracle's V-cycle and its residual restriction."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle.twogrid import TwoGrid
from paper_2104_01439_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# whole FGMRES solves (k, n, p) of the orders not in the batched case
SOLVES = [(14.0, 40, 2), (9.0, 16, 3)]

# (k, n, p, s, nu)
CASES = [(12.0, 64, 1, 1 + 0.5j, 2), (9.0, 46, 1, 1 + 0.4j, 1), (10.0, 36, 2, 1 + 0.5j, 2),
         (8.0, 18, 2, 1 + 0.6j, 3), (7.0, 10, 3, 1 + 0.5j, 2)]

CHILD = r"""
import os, sys
import numpy as np
import torch
sys.path.insert(0, ROOT)
from paper_2104_01439_amd import hz, inputs
out = {}
for i, (k, n, p, s, nu) in enumerate(CASES):
    print("[unfused] case", i, flush=True)
    pr = hz.Problem(k, 1.0 / n, p, s, nu=nu)
    f = torch.from_numpy(inputs.random_complex(pr.N, seed=50 + i)).cuda()
    x = torch.from_numpy(inputs.random_complex(pr.N, seed=60 + i)).cuda()
    for prec in ("fp64", "mixed"):
        out[f"v{i}_{prec}"] = pr.apply("VCYCLE", f, prec=prec).cpu().numpy()
        out[f"r{i}_{prec}"] = pr.apply("RESID_RESTRICT", x, f, prec=prec).cpu().numpy()
    pr.close()
print("[unfused] batched", flush=True)
pr = hz.Problem(12.0, 1 / 64, 1, 1 + 0.5j)
Fs = [pr.planewave_rhs(t) for t in (0.3, 1.9)]
us, rs = hz.solve_batched([pr], Fs, 2, tol=1e-9)
out["b0"], out["b1"] = us[0].cpu().numpy(), us[1].cpu().numpy()
out["bits"] = np.array([r["iterations"] for r in rs])
pr.close()
for q, (k, n, p) in enumerate(SOLVES):
    print("[unfused] solve", q, flush=True)
    pr = hz.Problem(k, 1.0 / n, p, 1 + 0.5j)
    u, r = pr.solve(pr.planewave_rhs(0.7), tol=1e-9, history=False)
    out[f"s{q}"], out[f"s{q}_its"] = u.cpu().numpy(), np.array(r["iterations"])
    pr.close()
kc = 30.0 * inputs.wedge_mu(32)
pr = hz.Problem.cells(kc, 1 + 1j * kc ** -0.5, 1 / 32, 1)
f = torch.from_numpy(inputs.random_complex(pr.N, seed=77)).cuda()
out["cells"] = pr.apply("VCYCLE", f).cpu().numpy()
pr.close()
np.savez(OUT, **out)
print("RESULT ok", flush=True)
"""


@pytest.fixture(scope="module")
def unfused(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("fused") / "unfused.npz")
    code = f"ROOT = {ROOT!r}\nCASES = {CASES!r}\nSOLVES = {SOLVES!r}\nOUT = {out!r}\n" + CHILD
    env = dict(os.environ, HZ_FUSE_PC="0", HZ_FUSE_RR="0")
    p = subprocess.run([sys.executable, "-u", "-c", code], env=env, capture_output=True,
                       text=True, timeout=240)
    print(p.stdout[-2000:], p.stderr[-2000:], flush=True)
    assert p.returncode == 0 and "RESULT ok" in p.stdout
    return dict(np.load(out))


@pytest.fixture(scope="module")
def hz():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2104_01439_amd import hz as h
    h.lib()
    return h


@pytest.mark.parametrize("i", range(len(CASES)))
def test_fused_vcycle_equals_two_pass(hz, unfused, i):
    import torch
    k, n, p, s, nu = CASES[i]
    print(f"[fused] case {i}: k={k} n={n} p={p} nu={nu}", flush=True)
    pr = hz.Problem(k, 1.0 / n, p, s, nu=nu)
    f = inputs.random_complex(pr.N, seed=50 + i)
    x = inputs.random_complex(pr.N, seed=60 + i)
    fd, xd = torch.from_numpy(f).cuda(), torch.from_numpy(x).cuda()
    tg = TwoGrid(k, n, p, s, nu=nu, omega=0.6)
    ref = tg.vcycle(f)
    ref_rr = tg.P.T @ (f - tg.Aeps @ x)
    for prec, tol, tol_rr in (("fp64", 1e-10, 1e-12), ("mixed", 2e-6, 2e-6)):
        z = pr.apply("VCYCLE", fd, prec=prec).cpu().numpy()
        assert np.array_equal(z, unfused[f"v{i}_{prec}"]), (i, prec)
        e = np.linalg.norm(z - ref) / np.linalg.norm(ref)
        assert e <= tol, (i, prec, e)
        rc = pr.apply("RESID_RESTRICT", xd, fd, prec=prec).cpu().numpy()
        assert np.array_equal(rc, unfused[f"r{i}_{prec}"]), (i, prec, "resid_restrict")
        e = np.linalg.norm(rc - ref_rr) / np.linalg.norm(ref_rr)
        assert e <= tol_rr, (i, prec, "resid_restrict", e)
    pr.close()


def test_fused_batched_solve_equals_two_pass(hz, unfused):
    pr = hz.Problem(12.0, 1 / 64, 1, 1 + 0.5j)
    Fs = [pr.planewave_rhs(t) for t in (0.3, 1.9)]
    us, rs = hz.solve_batched([pr], Fs, 2, tol=1e-9)
    assert [r["iterations"] for r in rs] == list(unfused["bits"])
    assert np.array_equal(us[0].cpu().numpy(), unfused["b0"])
    assert np.array_equal(us[1].cpu().numpy(), unfused["b1"])
    pr.close()


@pytest.mark.parametrize("q", range(len(SOLVES)))
def test_fused_solve_equals_two_pass(hz, unfused, q):
    k, n, p = SOLVES[q]
    pr = hz.Problem(k, 1.0 / n, p, 1 + 0.5j)
    u, r = pr.solve(pr.planewave_rhs(0.7), tol=1e-9, history=False)
    assert r["iterations"] == int(unfused[f"s{q}_its"])
    assert np.array_equal(u.cpu().numpy(), unfused[f"s{q}"])
    pr.close()


def test_per_point_operator_keeps_two_pass(hz, unfused):
    import torch
    kc = 30.0 * inputs.wedge_mu(32)
    pr = hz.Problem.cells(kc, 1 + 1j * kc ** -0.5, 1 / 32, 1)
    f = torch.from_numpy(inputs.random_complex(pr.N, seed=77)).cuda()
    assert np.array_equal(pr.apply("VCYCLE", f).cpu().numpy(), unfused["cells"])
    pr.close()
