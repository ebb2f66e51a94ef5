"""Short fixed workload for kernel profilers (rocprofv3 --kernel-trace / --pmc).

Creates one problem of a named workload (its creation runs the coarse factorisation), then
runs, each on torch's current stream:
  * `--copy-mib` MiB of a plain FP64 scale y = 1.0 * x (a copy-shaped kernel of known
    size: reads and writes exactly that many bytes), the calibration for HBM counters;
  * `--applies` applications of A_0 (matrix-free fine stencil, 32 B per fine dof);
  * `--stencils` applications of each other fine-level pass of the V-cycle (Jacobi sweep,
    residual + restriction, restriction, prolongation);
  * `--coarse-solves` coarse direct solves (multifrontal: every stored factor entry read
    once; bytes per system from the problem's own counters);
  * `--vcycles` whole V-cycles (their fine passes include the post-smoothing sweep that
    stages the coarse-grid correction itself).
It prints the device time of each group from HIP events and the algorithmic bytes, so that
counter totals can be set against them:

    python3 -m paper_2104_01439_amd.profile_run --workload p1_k400_n2048
"""

import argparse
import json
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="p1_k400_n2048")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--applies", type=int, default=8)
    ap.add_argument("--coarse-solves", type=int, default=4)
    ap.add_argument("--stencils", type=int, default=0)
    ap.add_argument("--vcycles", type=int, default=0)
    a = ap.parse_args(argv)

    import torch
    from paper_2104_01439_amd import hz, inputs
    from paper_2104_01439_amd.roofline import stencil_apply_bytes

    cfgs = {c["name"]: c for c in (inputs.CFG_SMALL, inputs.CFG_P1_LARGE, inputs.CFG_MIXED,
                                   inputs.CFG_SWEEP)}
    cfg = cfgs[a.workload]
    torch.cuda.set_device(0)
    k, n, p = cfg["k"], cfg["n"], cfg["p"]
    s = cfg.get("s", 1 + 0.5j)
    pr = hz.Problem(k, 1.0 / n, p, s, nu=cfg["nu"], omega=cfg["omega"], restart=cfg["restart"],
                    prec=a.prec, timing=True)
    F = pr.planewave_rhs(cfg.get("theta", 0.0))
    out = {"workload": cfg["name"], "prec": a.prec, "n_dofs": pr.N, "n_coarse": pr.Nc}

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()                                    # warm
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / max(reps, 1)

    nel = a.copy_mib * (1 << 20) // 8
    x = torch.ones(nel, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    ms = timed(lambda: torch.mul(x, 1.0, out=y), 4)
    out["copy"] = {"bytes_read": nel * 8, "bytes_written": nel * 8, "ms": ms,
                   "GB/s": 2 * nel * 8 / (ms * 1e-3) / 1e9}
    del x, y

    if a.applies:
        ms = timed(lambda: pr.apply("A0", F, prec=a.prec), a.applies)
        b = stencil_apply_bytes(n, p)
        out["A0"] = {"bytes": b, "ms": ms, "GB/s": b / (ms * 1e-3) / 1e9}
    if a.stencils:
        from paper_2104_01439_amd import inputs as inp
        x = torch.from_numpy(inp.random_complex(pr.N, seed=5)).cuda()
        f = torch.from_numpy(inp.random_complex(pr.N, seed=6)).cuda()
        xc = torch.from_numpy(inp.random_complex(pr.Nc, seed=7)).cuda()
        for op, arg in (("JACOBI", x), ("RESID_RESTRICT", x), ("RESTRICT", x), ("PROLONG", xc)):
            ms = timed(lambda: pr.apply(op, arg, f, prec=a.prec), a.stencils)
            out[op] = {"ms": ms}
    if a.vcycles:
        ms = timed(lambda: pr.apply("VCYCLE", F, prec=a.prec), a.vcycles)
        out["VCYCLE"] = {"ms": ms}
    if a.coarse_solves:
        rc = pr.apply("RESTRICT", F)
        pr.stats(reset=True)
        ms = timed(lambda: pr.apply("COARSE_SOLVE", rc, prec=a.prec), a.coarse_solves)
        st = pr.stats()
        b = st["coarse_bytes"] / max(st["coarse_systems"], 1)
        out["coarse_solve"] = {"bytes": b, "ms": ms, "GB/s": b / (ms * 1e-3) / 1e9,
                               "launches_per_system": st["coarse_solves"] / max(st["coarse_systems"], 1)}
    pr.close()
    del F
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
