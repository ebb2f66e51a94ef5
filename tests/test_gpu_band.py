"""The block-tridiagonal coarse factor (selected with HZ_COARSE=band; the multifrontal factor is
the default) against the oracle: the P3 k=200 h=1/256 coarse solve (blocks of 1155 columns,
two column passes of the persistent solve) against the stored oracle golden in FP64 and
with the FP32 factor, two right-hand sides per launch against one, and a whole FGMRES solve
against the oracle's. The library reads the switch once per process, so the checks run in a
child process."""

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, os, sys
import numpy as np
import torch
sys.path.insert(0, ROOT)
from paper_2104_01439_amd import hz, inputs
from oracle import Problem as OProblem
out = {}
g = dict(np.load(os.path.join(ROOT, "tests", "golden", "coarse_p3_k200_n256.npz")))
def errs(x):
    xi = x[g["idx"]]
    e_s = np.linalg.norm(xi - g["y_idx"]) / np.linalg.norm(g["y_idx"])
    e_n = abs(np.linalg.norm(x) - g["y_norm"]) / g["y_norm"]
    proj = np.array([np.vdot(inputs.random_complex(x.size, seed=int(g["proj_seed"]) + i), x)
                     for i in range(len(g["proj"]))])
    return max(e_s, e_n, float(np.max(np.abs(proj - g["proj"])) / np.max(np.abs(g["proj"]))))
for prec in ("fp64", "mixed"):
    print("[band] P3 n=256", prec, flush=True)
    pr = hz.Problem(200.0, 1 / 256, 3, 1 + 0.5j, prec=prec)
    r = torch.from_numpy(inputs.random_complex(pr.Nc, seed=int(g["rhs_seed"]))).cuda()
    y = pr.apply("COARSE_SOLVE", r, prec=prec)
    Fs = [pr.planewave_rhs(t) for t in (0.3, 2.2)]
    us, rs = hz.solve_batched([pr], Fs, 2, tol=1e-6)
    same = True
    for q in range(2):
        u1, r1 = pr.solve(Fs[q], tol=1e-6, history=False)
        same = same and r1["iterations"] == rs[q]["iterations"] and bool(torch.equal(u1, us[q]))
    out[prec] = {"golden": errs(y.cpu().numpy()), "batched_equals_single": same}
    pr.close()
print("[band] FGMRES P1 k=16 n=64", flush=True)
op = OProblem(16.0, 64, 1, 1 + 0.5j)
F = op.planewave_rhs(np.pi / 7)
ro = op.solve(F, tol=1e-10)
pr = hz.Problem(16.0, 1 / 64, 1, 1 + 0.5j)
u, r = pr.solve(torch.from_numpy(F).cuda(), tol=1e-10)
out["solve"] = {"iterations": r["iterations"], "oracle_iterations": ro["iterations"],
                "u_err": float(np.linalg.norm(u.cpu().numpy() - ro["u"]) / np.linalg.norm(ro["u"]))}
pr.close()
print("RESULT " + json.dumps(out), flush=True)
"""


def test_band_path_against_oracle():
    env = dict(os.environ, HZ_COARSE="band")
    code = "ROOT = " + repr(ROOT) + "\n" + CHILD
    p = subprocess.run([sys.executable, "-u", "-c", code], env=env, capture_output=True,
                       text=True, timeout=240)
    print(p.stdout[-2000:], p.stderr[-2000:], flush=True)
    assert p.returncode == 0
    res = json.loads(p.stdout.split("RESULT ", 1)[1])
    # measured: FP64 2.2e-13, FP32 factor 1.4e-7 (bounds as for the default factor)
    assert res["fp64"]["golden"] <= 1e-10
    assert res["mixed"]["golden"] <= 2e-6
    assert res["fp64"]["batched_equals_single"] and res["mixed"]["batched_equals_single"]
    assert abs(res["solve"]["iterations"] - res["solve"]["oracle_iterations"]) <= 1
    assert res["solve"]["u_err"] <= 1e-8
