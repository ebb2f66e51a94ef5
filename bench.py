#!/usr/bin/env python3
"""Benchmark: FGMRES solves/s of the twogrid-preconditioned Helmholtz solver on one MI355X.

One step = the whole path for one plane-wave problem: create_problem (stencil tables,
coarse assembly and block factorisation on the device), plane-wave load vector, FGMRES
solve to the configured tolerance, destroy. Inputs are synthetic (plane-wave impedance
data); nothing is read from disk. Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def coarse_solve_bytes(n, p, itemsize=16):
    """Algorithmic bytes of one coarse solve: every stored block inverse read twice
    (forward and backward sweep), plus the coarse right-hand side and solution."""
    nc = n // 2
    Mc = p * nc + 1
    blocks = nc * (p * Mc) ** 2 + Mc ** 2
    bwd = blocks - Mc ** 2          # the last block is read in the forward sweep only
    return (blocks + bwd) * itemsize + 3 * Mc * Mc * itemsize


def run_gpu(cfg, steps, warmup, prec):
    import torch
    from paper_2104_01439_amd import hz

    torch.cuda.set_device(0)
    k, n, p, s, th, tol = cfg["k"], cfg["n"], cfg["p"], cfg["s"], cfg["theta"], cfg["tol"]
    info = {}

    def step():
        pr = hz.Problem(k, 1.0 / n, p, s, nu=cfg["nu"], omega=cfg["omega"],
                        restart=cfg["restart"], tol=tol, prec=prec)
        F = pr.planewave_rhs(th)
        u, r = pr.solve(F, tol=tol, prec=prec, history=False)
        info.update(r)
        info["footprint_bytes"] = pr.info()["footprint_bytes"]
        pr.close()
        return r

    for i in range(warmup):
        r = step()
        log(f"warmup {i}: {r['iterations']} iterations, converged={r['converged']}, "
            f"setup {r['setup_s']:.3f}s solve {r['solve_s']:.3f}s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for i in range(steps):
        r = step()
        its.append(r["iterations"])
        log(f"step {i}: {r['iterations']} iterations, converged={r['converged']}, "
            f"setup {r['setup_s']:.3f}s solve {r['solve_s']:.3f}s")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # Dominant kernel: the coarse block triangular solves. Time repeated coarse solves on
    # the solve stream with HIP events; bytes are the algorithmic factor reads.
    pr = hz.Problem(k, 1.0 / n, p, s, nu=cfg["nu"], omega=cfg["omega"],
                    restart=cfg["restart"], tol=tol, prec=prec)
    x = torch.randn(pr.Nc, dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream()
    pr.apply("COARSE_SOLVE", x, prec=prec)
    reps = 5
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        pr.apply("COARSE_SOLVE", x, prec=prec)
    e1.record(stream)
    torch.cuda.synchronize()
    cs_ms = e0.elapsed_time(e1) / reps
    pr.close()
    item = 8 if prec == "mixed" else 16
    cs_bytes = coarse_solve_bytes(n, p, item)
    return dict(seconds=dt, iterations=its, info=info, coarse_ms=cs_ms, coarse_bytes=cs_bytes)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="p1_k400_n2048")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(independent solves shard across GPUs without communication; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)
    from paper_2104_01439_amd import inputs
    cfgs = {c["name"]: c for c in (inputs.CFG_SMALL, inputs.CFG_P1_LARGE, inputs.CFG_MIXED)}
    cfg = cfgs[a.workload]
    g = run_gpu(cfg, a.steps, a.warmup, a.prec)
    value = a.steps / g["seconds"]
    cs_gbs = g["coarse_bytes"] / (g["coarse_ms"] * 1e-3) / 1e9
    out = {
        "metric": "FGMRES solves/s",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * g["seconds"] / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if a.prec == "fp64" else "c64-precond/c128-outer",
        "data": "synthetic plane-wave impedance data",
        "config": {"workload": cfg["name"], "k": cfg["k"], "n": cfg["n"], "p": cfg["p"],
                   "shift": str(cfg["s"]), "tol": cfg["tol"], "restart": cfg["restart"],
                   "nu": cfg["nu"], "omega": cfg["omega"], "precision": a.prec,
                   "iterations": g["iterations"]},
        "roofline": {"kernel": "coarse block triangular solve", "bound": "hbm",
                     "achieved": cs_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": cs_gbs / HBM_PEAK_GBS, "traffic": None},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
