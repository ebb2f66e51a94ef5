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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2104_01439_amd.roofline import (FP64_MFMA_PEAK_TFLOPS, HBM_PEAK_GBS,  # noqa: E402
                                           STENCIL_BYTES_PER_DOF, coarse_solve_bytes,
                                           factor_bytes, factor_flops)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(path="profiles/k_mf_solve_p1_k400_n2048_traffic.txt"):
    """HBM bytes per coarse system of the multifrontal solve from the committed counter
    summary, or None when the kernel source has changed since the counters were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, path)) as f:
            kv = dict(l.split(": ", 1) for l in f.read().splitlines() if ": " in l and not l.startswith(" "))
        src = os.path.join(ROOT, kv["kernel_source"].strip())
        with open(src, "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()[:16]
        if h != kv["kernel_source_sha256_16"].strip():
            return None
        return float(kv["traffic_bytes_per_system"])
    except (OSError, KeyError, ValueError):
        return None


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return model, ncpu


def cpu_baseline_both(cfg, iterations):
    """The oracle's projected solve rate with its default threads (threaded BLAS in the
    banded LU and the dense products; the sparse products are single-threaded) and again
    limited to one thread."""
    from threadpoolctl import threadpool_limits
    allc = cpu_baseline(cfg, iterations)
    with threadpool_limits(limits=1):
        one = cpu_baseline(cfg, iterations)
    model, ncpu = host_cpu()
    allc["cpu_model"] = model
    allc["nproc"] = ncpu
    allc["one_thread"] = {"value": one["value"], "unit": one["unit"], "cores": 1,
                          "projected_s_per_solve": one["projected_s_per_solve"],
                          "sample_wall_s": one["sample_wall_s"]}
    return allc


def stencil_rates(cfg, prec, reps=20):
    """Live device time of each fine-level pass of the V-cycle at the workload's size (HIP
    events on the launch stream, `reps` back-to-back launches after a warm-up that also lets
    the tile autotuner settle), against its algorithmic bytes."""
    import torch
    from paper_2104_01439_amd import hz, inputs

    k, n, p, s = cfg["k"], cfg["n"], cfg["p"], cfg["s"]
    pr = hz.Problem(k, 1.0 / n, p, s, nu=cfg["nu"], omega=cfg["omega"], prec=prec)
    x = torch.from_numpy(inputs.random_complex(pr.N, seed=5)).cuda()
    f = torch.from_numpy(inputs.random_complex(pr.N, seed=6)).cuda()
    xc = torch.from_numpy(inputs.random_complex(pr.Nc, seed=7)).cuda()
    yf, yc = pr.empty(), pr.empty(coarse=True)
    B = STENCIL_BYTES_PER_DOF
    item = 16 if prec == "fp64" else 8
    passes = {
        "A0 apply": ("A0", x, None, yf, B["a0_apply"], 1),
        "Jacobi sweep": ("JACOBI", x, f, yf, B["jacobi_sweep"], 1),
        # P1: one pass (the residual is never stored); otherwise the two passes
        ("residual + restriction (one pass)" if p == 1 else "residual + restriction (2 kernels)"):
            ("RESID_RESTRICT", x, f, yc,
             B["resid_restrict_fused"] if p == 1 else B["residual"] + B["restriction"],
             1 if p == 1 else 2),
        "restriction": ("RESTRICT", x, None, yc, B["restriction"], 1),
        "prolongation": ("PROLONG", xc, None, yf, B["prolongation"], 1),
    }
    out = {}
    # on-box copy probe: torch's FP64 copy of 1 GiB (1 GiB read, 1 GiB written)
    xs = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    ys = torch.empty_like(xs)
    for _ in range(3):
        ys.copy_(xs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ys.copy_(xs)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * xs.numel() * 8 / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    del xs, ys
    out["copy probe (torch, 1 GiB)"] = {"GB/s": copy_gbs, "frac": copy_gbs / HBM_PEAK_GBS}
    for name, (op, a, b, y, bpd, nk) in passes.items():
        for _ in range(3):
            pr.apply(op, a, b, y=y, prec=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            pr.apply(op, a, b, y=y, prec=prec)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = bpd * (item / 16) * pr.N / (ms * 1e-3) / 1e9
        out[name] = {"us": 1e3 * ms, "bytes_per_dof": bpd * item / 16, "kernels": nk,
                     "GB/s": gbs, "frac": gbs / HBM_PEAK_GBS, "of_copy_probe": gbs / copy_gbs}
    pr.close()
    return out


def cpu_baseline(cfg, iterations):
    """The oracle (plain NumPy/SciPy FP64) timed on the host on a bounded sample of this
    workload and projected to one full solve.

    Sample: the fine-level work (setup, one V-cycle without its coarse solve, one A_0
    apply, one CGS2 step at j = 25) on the same plane-wave problem at n = 512 (k scaled to
    keep k h), scaled by the fine-dof ratio; the banded coarse LU (LAPACK zgbtrf/zgbtrs) on
    the leading 128 lattice rows of the real coarse operator (full bandwidth), scaled by the
    row ratio; iterations = the GPU solve's count (the two agree within one iteration on
    every size the parity tests compare).
    """
    import numpy as np
    from oracle import Problem as OProblem
    from oracle.fem import Discretisation
    from oracle.twogrid import BandedLU
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    n, p, k, s = cfg["n"], cfg["p"], cfg["k"], cfg["s"]
    ns = min(n, 512)
    ks = k * ns / n
    t0 = time.perf_counter()
    t = time.perf_counter()
    pr = OProblem(ks, ns, p, s, nu=cfg["nu"], omega=cfg["omega"])
    t_setup_s = time.perf_counter() - t
    F = pr.planewave_rhs(cfg["theta"])
    v = F / np.linalg.norm(F)
    reps = 3
    t = time.perf_counter()
    for _ in range(reps):
        z = pr.tg.vcycle(v)
    t_vc = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    for _ in range(reps):
        pr.tg.coarse_solve(pr.tg.restrict_residual(np.zeros_like(v), v))
    t_cs_s = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    for _ in range(reps):
        w = pr.apply_A0(z)
    t_a0 = (time.perf_counter() - t) / reps
    V = np.random.default_rng(0).standard_normal((26, pr.N)) + 0j
    t = time.perf_counter()
    for _ in range(reps):
        x = w
        for _ in range(2):
            hh = V.conj() @ x
            x = x - V.T @ hh
    t_cgs = (time.perf_counter() - t) / reps
    scale_f = ((p * n + 1) / (p * ns + 1)) ** 2
    # coarse band strip of the full-size problem
    dc = Discretisation(n // 2, p)
    t = time.perf_counter()
    Ac = dc.operator(k, s)
    t_asm = time.perf_counter() - t
    rows = min(128, dc.M)
    m = rows * dc.M
    t = time.perf_counter()
    lu = BandedLU(Ac[:m, :m])
    t_fac = time.perf_counter() - t
    t = time.perf_counter()
    lu.solve(np.ones(m, complex))
    t_sol = time.perf_counter() - t
    scale_c = dc.M / rows
    setup = t_setup_s * scale_f + t_asm + t_fac * scale_c
    per_it = (t_vc - t_cs_s + t_a0 + t_cgs) * scale_f + t_sol * scale_c
    total = setup + iterations * per_it
    wall = time.perf_counter() - t0
    return {"value": 1.0 / total, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
            "projected_s_per_solve": total, "sample_wall_s": wall,
            "sample": (f"oracle fine-level setup/V-cycle/A0/CGS2(j=25) at n={ns} (k={ks:g}) "
                       f"x{scale_f:.1f} fine dofs; banded LU factor+solve on {rows} of "
                       f"{dc.M} coarse lattice rows (bandwidth {lu.kl}) x{scale_c:.1f}; "
                       f"{iterations} iterations (GPU count); projected, not a full run")}


def run_gpu(cfg, steps, warmup, prec):
    import torch
    from paper_2104_01439_amd import hz

    torch.cuda.set_device(0)
    k, n, p, s, th, tol = cfg["k"], cfg["n"], cfg["p"], cfg["s"], cfg["theta"], cfg["tol"]
    info = {}

    stats = []

    def step(record=False):
        pr = hz.Problem(k, 1.0 / n, p, s, nu=cfg["nu"], omega=cfg["omega"],
                        restart=cfg["restart"], tol=tol, prec=prec, timing=True)
        F = pr.planewave_rhs(th)
        u, r = pr.solve(F, tol=tol, prec=prec, history=False)
        info.update(r)
        info["footprint_bytes"] = pr.info()["footprint_bytes"]
        if record:
            stats.append(pr.stats())
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
        r = step(record=True)
        its.append(r["iterations"])
        log(f"step {i}: {r['iterations']} iterations, converged={r['converged']}, "
            f"setup {r['setup_s']:.3f}s solve {r['solve_s']:.3f}s")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # Dominant kernel: the multifrontal coarse solve (k_mf_sub for the bottom subtrees and
    # k_mf_solve for each higher tree height, per pass). Device time from HIP event pairs
    # around every coarse solve on the solve stream during the timed steps; bytes are the
    # algorithmic factor and vector traffic. Unit: one coarse system (all its launches).
    systems = sum(x["coarse_systems"] for x in stats)
    launches = sum(x["coarse_solves"] for x in stats)
    cs_ms = sum(x["coarse_solve_ms"] for x in stats) / max(systems, 1)
    factor_ms = sum(x["factor_ms"] for x in stats) / max(len(stats), 1)
    factor_flop = sum(x["factor_flop"] for x in stats) / max(len(stats), 1)
    cs_bytes = sum(x["coarse_bytes"] for x in stats) / max(systems, 1)
    return dict(seconds=dt, iterations=its, info=info, coarse_ms=cs_ms, coarse_bytes=cs_bytes,
                coarse_systems=systems, launches_per_system=launches / max(systems, 1),
                factor_ms=factor_ms, factor_flop=factor_flop)


def near_optimal_beta(betas, its, rhos):
    """argmin over beta of the mean iteration count over the right-hand sides; ties broken by
    the smaller mean convergence factor, then by the smaller beta."""
    keys = [(float(np.mean(its[i])), float(np.mean(rhos[i])), betas[i]) for i in range(len(betas))]
    return min(keys)[2]


def run_sweep(cfg, steps, warmup, prec):
    """The shift sweep: every beta with every incidence angle, the right-hand sides of one
    shift and several shifts in one lockstep batch; groups of shifts sized to HBM."""
    import torch
    from paper_2104_01439_amd import hz, inputs

    torch.cuda.set_device(0)
    k, n, p, tol = cfg["k"], cfg["n"], cfg["p"], cfg["tol"]
    betas, thetas = inputs.sweep_betas(), inputs.sweep_thetas()
    nr = len(thetas)
    free, _ = torch.cuda.mem_get_info()
    item = 8 if prec == "mixed" else 16
    per_shift = factor_bytes(n, p, item) + hz.batch_workspace_bytes(1.0 / n, p, 1, nr, prec=prec,
                                                                    restart=cfg["restart"])
    gmax = max(1, int(0.85 * (free - 2 * factor_bytes(n, p)) // per_shift))
    ngroups = -(-len(betas) // gmax)
    gsize = -(-len(betas) // ngroups)
    log(f"sweep: {len(betas)} shifts x {nr} angles, groups of {gsize} shifts "
        f"({per_shift / 1e9:.2f} GB per shift, {free / 1e9:.0f} GB free)")

    # the coarse factorisations of a group are independent and latency-bound: several run at
    # once, each from its own host thread on its own stream
    from concurrent.futures import ThreadPoolExecutor
    nsetup = 8
    streams = [torch.cuda.Stream() for _ in range(nsetup)]

    def create(ib):
        i, b = ib
        torch.cuda.set_device(0)
        with torch.cuda.stream(streams[i % nsetup]):
            return hz.Problem(k, 1.0 / n, p, 1 + 1j * b, nu=cfg["nu"], omega=cfg["omega"],
                              restart=cfg["restart"], tol=tol, prec=prec, timing=True)

    def sweep(record):
        its = [[0] * nr for _ in betas]
        rhos = [[0.0] * nr for _ in betas]
        stats, setup_s, conv = [], 0.0, True
        Fs = None
        for g0 in range(0, len(betas), gsize):
            gb = betas[g0:g0 + gsize]
            t = time.perf_counter()
            with ThreadPoolExecutor(nsetup) as ex:
                probs = list(ex.map(create, enumerate(gb)))
            torch.cuda.synchronize()
            setup_s += time.perf_counter() - t
            if Fs is None:
                Fs = [probs[0].planewave_rhs(th) for th in thetas]   # independent of the shift
            t = time.perf_counter()
            us, rs = hz.solve_batched(probs, [F for _ in gb for F in Fs], nr, tol=tol)
            gi = [x["iterations"] for x in rs]
            log(f"  shifts beta {gb[0]:.3f}..{gb[-1]:.3f}: iterations {min(gi)}..{max(gi)}, "
                f"batched solve {time.perf_counter() - t:.2f}s")
            for i in range(len(gb)):
                for r in range(nr):
                    x = rs[i * nr + r]
                    its[g0 + i][r] = x["iterations"]
                    rhos[g0 + i][r] = x["rel_res_true"] ** (1.0 / max(x["iterations"], 1))
                    conv = conv and bool(x["converged"])
            if record:
                stats += [pr.stats() for pr in probs]
            for pr in probs:
                pr.close()
            del us
        return its, rhos, stats, setup_s, conv

    for i in range(warmup):
        sweep(False)
        log(f"warmup {i} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        its, rhos, stats, setup_s, conv = sweep(True)
        log(f"sweep {i}: mean iterations {np.mean(its):.1f}, setup {setup_s:.2f}s, "
            f"converged={conv}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    bstar = near_optimal_beta(betas, its, rhos)
    systems = sum(x["coarse_systems"] for x in stats)
    launches = sum(x["coarse_solves"] for x in stats)
    cs_ms = sum(x["coarse_solve_ms"] for x in stats) / max(systems, 1)
    vcyc = sum(x["vcycles"] for x in stats)
    return dict(seconds=dt, solves=steps * len(betas) * nr, its=its, bstar=bstar,
                sigma=2 + math.log(bstar) / math.log(k), group=gsize, setup_s=setup_s,
                coarse_ms=cs_ms, coarse_systems=systems, launches_per_system=launches / max(systems, 1),
                coarse_bytes=sum(x["coarse_bytes"] for x in stats) / max(systems, 1),
                factor_ms=sum(x["factor_ms"] for x in stats) / max(len(stats), 1),
                betas=betas, thetas=thetas, converged=conv)


def run_serving(count, rate, prec, max_active, tol=1e-8, restart=50):
    """The serving stream: requests arrive at their (seeded) times, the engine admits them by
    memory and slots and solves them with continuous batching; latency = submission to
    completion."""
    import torch
    from paper_2104_01439_amd import hz, inputs

    torch.cuda.set_device(0)
    reqs = inputs.serving_requests(count, seed=1, rate=rate)
    # the clients' solution buffers exist before the engine sizes its budget from free memory
    us = [torch.empty((r["p"] * r["n"] + 1) ** 2, dtype=torch.complex128, device="cuda")
          for r in reqs]
    eng = hz.Engine(max_active=max_active, setup_threads=4, tol=tol, restart=restart, prec=prec)
    done = {}
    t0 = time.perf_counter()
    nxt = 0
    last_log = t0
    while len(done) < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(reqs) and reqs[nxt]["t"] <= now:
            r = reqs[nxt]
            eng.submit(r["id"], r["k"], 1.0 / r["n"], r["p"], 1 + 1j * r["beta"], theta=r["theta"],
                       u=us[nxt])
            nxt += 1
        wait = 200 if nxt >= len(reqs) else max(1, int(1e3 * (reqs[nxt]["t"] - now)))
        for d, u in eng.poll(wait_ms=min(wait, 200)):
            done[d["id"]] = d
        if time.perf_counter() - last_log > 20:
            last_log = time.perf_counter()
            inf = eng.info()
            free = torch.cuda.mem_get_info()[0]
            log(f"  serving: {len(done)}/{len(reqs)} done, {inf['admitted']} admitted, "
                f"{inf['queued']} queued, {inf['bytes_in_use'] / 1e9:.1f} GB in use, "
                f"{free / 1e9:.1f} GB free on the device")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    eng.close()
    lat = np.array([done[r["id"]]["latency_s"] for r in reqs])
    its = np.array([done[r["id"]]["iterations"] for r in reqs])
    ok = all(done[r["id"]]["status"] == 0 and done[r["id"]]["converged"] == 1 for r in reqs)
    worst = max(done[r["id"]]["rel_res_true"] for r in reqs)
    return dict(seconds=dt, solves=len(reqs), p50=float(np.percentile(lat, 50)),
                p99=float(np.percentile(lat, 99)), mean_its=float(its.mean()), ok=ok,
                worst_rel_res=worst, classes=sorted({(r["p"], r["n"]) for r in reqs}))


def run_sequential_fp64(count, tol=1e-8, restart=50):
    """The plain FP64 path on the same requests, one after the other (create, solve, free)."""
    import torch
    from paper_2104_01439_amd import hz, inputs

    torch.cuda.set_device(0)
    reqs = inputs.serving_requests(count, seed=1, rate=None)
    t0 = time.perf_counter()
    last_log = t0
    worst, ok = 0.0, True
    for i, r in enumerate(reqs):
        pr = hz.Problem(r["k"], 1.0 / r["n"], r["p"], 1 + 1j * r["beta"], tol=tol, restart=restart)
        _, res = pr.solve(pr.planewave_rhs(r["theta"]), tol=tol, history=False)
        worst = max(worst, res["rel_res_true"])
        ok = ok and bool(res["converged"])
        pr.close()
        if time.perf_counter() - last_log > 20:
            last_log = time.perf_counter()
            log(f"  plain fp64: {i + 1}/{len(reqs)} done")
    torch.cuda.synchronize()
    return dict(seconds=time.perf_counter() - t0, solves=len(reqs), worst_rel_res=worst, ok=ok)


def run_precision(cfg, steps, warmup):
    """FP64 and mixed-precision solves of the same problem on the GPU; the oracle checks both
    on a reduced mesh of the same resolution (k h / p fixed) where it finishes in seconds."""
    import torch
    from paper_2104_01439_amd import hz
    from oracle import Problem as OProblem

    torch.cuda.set_device(0)
    k, n, p, s, th, tol = cfg["k"], cfg["n"], cfg["p"], cfg["s"], cfg["theta"], cfg["tol"]
    out = {}
    sols = {}
    for prec in ("fp64", "mixed"):
        times, its = [], []
        for i in range(warmup + steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            pr = hz.Problem(k, 1.0 / n, p, s, nu=cfg["nu"], omega=cfg["omega"],
                            restart=cfg["restart"], tol=tol, prec=prec)
            u, r = pr.solve(pr.planewave_rhs(th), tol=tol, history=False)
            torch.cuda.synchronize()
            if i >= warmup:
                times.append(time.perf_counter() - t)
                its.append(r["iterations"])
            pr.close()
            log(f"{prec} step {i}: {r['iterations']} iterations, {time.perf_counter() - t:.2f}s")
        sols[prec] = u
        out[prec] = {"solves_s": len(times) / sum(times), "iterations": its,
                     "true_rel_res": r["rel_res_true"]}
    d = (sols["mixed"] - sols["fp64"]).norm().item() / sols["fp64"].norm().item()
    out["iteration_delta"] = out["mixed"]["iterations"][0] - out["fp64"]["iterations"][0]
    out["rel_diff_mixed_vs_fp64"] = d
    # oracle on the reduced mesh
    ns = 64
    ks = k * ns / n
    op = OProblem(ks, ns, p, s, nu=cfg["nu"], omega=cfg["omega"])
    F = op.planewave_rhs(th)
    ro = op.solve(F, tol=tol, m=cfg["restart"])
    chk = {"k": ks, "n": ns, "p": p, "oracle_iterations": ro["iterations"]}
    for prec in ("fp64", "mixed"):
        pr = hz.Problem(ks, 1.0 / ns, p, s, nu=cfg["nu"], omega=cfg["omega"],
                        restart=cfg["restart"], prec=prec)
        u, r = pr.solve(torch.from_numpy(F).cuda(), tol=tol, history=False)
        uo = u.cpu().numpy()
        chk[prec] = {"iterations": r["iterations"],
                     "u_rel_err_vs_oracle": float(np.linalg.norm(uo - ro["u"]) / np.linalg.norm(ro["u"]))}
        pr.close()
    out["oracle_check"] = chk
    return out


def main_precision(a, cfg):
    g = run_precision(cfg, a.steps, a.warmup)
    value = g["mixed"]["solves_s"]
    out = {
        "metric": "FGMRES solves/s",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 / value,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-precond/f64-outer",
        "data": "synthetic plane-wave impedance data",
        "config": {"workload": cfg["name"], "k": cfg["k"], "n": cfg["n"], "p": cfg["p"],
                   "shift": str(cfg["s"]), "tol": cfg["tol"], "restart": cfg["restart"],
                   "nu": cfg["nu"], "omega": cfg["omega"], "precision": "mixed vs fp64"},
        "precision": g,
        "speedup_mixed_vs_fp64": value / g["fp64"]["solves_s"],
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main_serving_plain(a):
    """The plain FP64 path alone on the serving stream's requests, one after the other."""
    sq = run_sequential_fp64(a.requests)
    value = sq["solves"] / sq["seconds"]
    out = {"metric": "FGMRES solves/s", "value": value, "unit": "solves/s", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": 1e3 * sq["seconds"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic plane-wave impedance data",
           "config": {"workload": "serving_stream_plain_fp64_sequential", "requests": a.requests,
                      "seed": 1, "tol": 1e-8, "restart": 50},
           "worst_true_rel_res": sq.get("worst_rel_res"), "all_converged": sq.get("ok"),
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def main_serving(a):
    if a.plain_only:
        return main_serving_plain(a)
    g = run_serving(a.requests, a.rate if a.rate > 0 else None, a.prec, a.max_active)
    value = g["solves"] / g["seconds"]
    out = {
        "metric": "FGMRES solves/s",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": 1e3 * g["seconds"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.prec == "fp64" else "f32-precond/f64-outer",
        "data": "synthetic plane-wave impedance data",
        "config": {"workload": "serving_stream", "requests": a.requests,
                   "arrivals": "saturated (all at t=0)" if a.rate <= 0 else f"Poisson {a.rate}/s",
                   "seed": 1, "tol": 1e-8, "restart": 50, "precision": a.prec,
                   "max_active": a.max_active, "classes": [list(c) for c in g["classes"]]},
        "latency_s": {"p50": g["p50"], "p99": g["p99"]},
        "mean_iterations": g["mean_its"],
        "all_converged": g["ok"],
        "worst_true_rel_res": g["worst_rel_res"],
        "roofline": None,
        "cpu_baseline": None,
    }
    if a.baseline:
        log("plain FP64 path, sequential, same requests ...")
        sq = run_sequential_fp64(a.requests)
        out["plain_fp64_sequential"] = {"value": sq["solves"] / sq["seconds"], "unit": "solves/s",
                                        "seconds": sq["seconds"]}
        out["speedup_vs_plain_fp64"] = value / out["plain_fp64_sequential"]["value"]
    print(json.dumps(out), flush=True)


def main_search(a):
    """Shift-search samples (Sec. 5 data generation) on the GPU: samples/s, the data set, the
    Table 1 map's exponents beside the searched ones, and a per-order refit of the map."""
    import torch
    from paper_2104_01439_amd import inputs, samplegen, shiftmap

    torch.cuda.set_device(0)
    samples = inputs.shift_samples(a.samples, seed=2, ells=tuple(range(4, a.max_ell + 1)))
    log(f"shift search: {len(samples)} samples, ell 4..{a.max_ell} ...")
    for i in range(a.warmup):
        samplegen.generate(samples[:4])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rows = samplegen.generate(samples)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    evals = sum(r["evaluations"] for r in rows)
    tab = [float(shiftmap.sigma_map(r["k"], r["ell"], r["p"])) for r in rows]
    fits = {}
    for p in (1, 2, 3):
        sel = [r for r in rows if r["p"] == p]
        if len(sel) < 4:
            continue
        w = shiftmap.sample_weights([r["ell"] for r in sel], [p] * len(sel))
        est, loss = shiftmap.fit([r["k"] for r in sel], [r["ell"] for r in sel],
                                 [r["sigma_hat"] for r in sel], w, epochs=a.epochs)
        fits[p] = {"weights": est, "loss": loss, "samples": len(sel)}
    out = {
        "metric": "shift-search samples/s",
        "value": len(rows) / dt,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: random real right-hand sides, g = 0",
        "config": {"workload": "shift_search", "samples": len(rows), "ells": [4, a.max_ell],
                   "sigma_range": [1.0, 2.0], "tol": 1e-2, "solve_tol": 1e-8, "maxit": 50},
        "solves_per_s": evals / dt,
        "evaluations": evals,
        "rows": rows,
        "table1_sigma": tab,
        "mean_abs_sigma_hat_minus_table1": float(np.mean([abs(r["sigma_hat"] - t)
                                                           for r, t in zip(rows, tab)])),
        "refit": fits,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def pn_stencil_rates(pr, reps=20):
    """Live device time of the per-point (heterogeneous k) fine passes of a P1 problem, against
    their algorithmic bytes."""
    import torch
    from paper_2104_01439_amd import inputs
    from paper_2104_01439_amd.roofline import STENCIL_PN_BYTES_PER_DOF_P1 as B
    x = torch.from_numpy(inputs.random_complex(pr.N, seed=5)).cuda()
    f = torch.from_numpy(inputs.random_complex(pr.N, seed=6)).cuda()
    yf = pr.empty()
    out = {}
    for name, (op, b, bpd) in {"A0 apply": ("A0", None, B["a0_apply"]),
                               "Jacobi sweep": ("JACOBI", f, B["jacobi_sweep"])}.items():
        for _ in range(3):
            pr.apply(op, x, b, y=yf)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            pr.apply(op, x, b, y=yf)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = bpd * pr.N / (ms * 1e-3) / 1e9
        out[name] = {"us": 1e3 * ms, "bytes_per_dof": bpd, "GB/s": gbs, "frac": gbs / HBM_PEAK_GBS}
    return out


def main_wedge(a):
    """Heterogeneous wavenumber (Sec. 6 setting): the wedge profile k = k_max mu(x), the point
    source at (0.5, 0.55), g = 0, one problem per shift policy eps in {k, k^1.5, k^2,
    k^sigma_p(k)} applied per cell; FGMRES(50) to 1e-8, at most 500 iterations. value: solves/s
    with the map's shift."""
    import torch
    from paper_2104_01439_amd import hz, inputs, shiftmap

    torch.cuda.set_device(0)
    cfg = inputs.CFG_WEDGE
    n, p, h = cfg["n"], cfg["p"], 1.0 / cfg["n"]
    kc = cfg["kmax"] * inputs.wedge_mu(n)
    rows, stencils = {}, None
    for pol in ("k", "k1.5", "k2", "map"):
        sc = shiftmap.cell_shifts(kc, h, p, pol)
        log(f"wedge: policy {pol}: creating (P{p}, h = 1/{n}, k_max {cfg['kmax']}) ...")
        t0 = time.perf_counter()
        pr = hz.Problem.cells(kc, sc, h, p, nu=cfg["nu"], omega=cfg["omega"],
                              restart=cfg["restart"], maxit=500, tol=cfg["tol"], timing=True)
        setup = time.perf_counter() - t0
        F = pr.gaussian_rhs(cfg["source"])
        for _ in range(a.warmup):
            pr.solve(F, history=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            u, r = pr.solve(F, history=False)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
        st = pr.stats()
        rows[pol] = {"iterations": r["iterations"], "converged": r["converged"],
                     "rel_res_true": r["rel_res_true"], "setup_s": setup,
                     "factor_ms": st["factor_ms"], "solve_s": dt}
        log(f"  {r['iterations']} iterations, {dt:.3f} s per solve, set-up {setup:.2f} s")
        if pol == "map":
            stencils = pn_stencil_rates(pr)
        pr.close()
    m = rows["map"]
    out = {
        "metric": "FGMRES solves/s",
        "value": 1.0 / m["solve_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * m["solve_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic three-layer wedge profile, Gaussian point source, g = 0",
        "config": {"workload": cfg["name"], "kmax": cfg["kmax"], "n": n, "p": p,
                   "source": list(cfg["source"]), "tol": cfg["tol"], "restart": cfg["restart"],
                   "maxit": 500, "shift": "eps = k^sigma_p(k, ell) per cell"},
        "policies": rows,
        "stencil_passes_per_point": stencils,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    release()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="p1_k400_n2048")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "mixed", "compare"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--requests", type=int, default=200, help="serving: stream prefix length")
    ap.add_argument("--rate", type=float, default=0.0, help="serving: arrivals per s (0: all at once)")
    ap.add_argument("--max-active", type=int, default=32, help="serving: engine slots")
    ap.add_argument("--baseline", action="store_true", help="serving: also time the plain FP64 path")
    ap.add_argument("--plain-only", action="store_true", help="serving: time the plain FP64 path only")
    ap.add_argument("--samples", type=int, default=48, help="shift_search: samples")
    ap.add_argument("--max-ell", type=int, default=8, help="shift_search: largest mesh level")
    ap.add_argument("--epochs", type=int, default=20000, help="shift_search: refit epochs")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(independent solves shard across GPUs without communication; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)
    from paper_2104_01439_amd import inputs
    if a.workload == "serving":
        return main_serving(a)
    if a.workload == "shift_search":
        return main_search(a)
    if a.workload == inputs.CFG_WEDGE["name"]:
        return main_wedge(a)
    if a.workload == inputs.CFG_MIXED["name"] and a.prec == "compare":
        return main_precision(a, inputs.CFG_MIXED)
    if a.workload == inputs.CFG_SWEEP["name"]:
        return main_sweep(a, inputs.CFG_SWEEP)
    cfgs = {c["name"]: c for c in (inputs.CFG_SMALL, inputs.CFG_P1_LARGE, inputs.CFG_MIXED)}
    cfg = cfgs[a.workload]
    g = run_gpu(cfg, a.steps, a.warmup, a.prec)
    value = a.steps / g["seconds"]
    log("fine-level passes: live timing at the workload's size ...")
    stencils = stencil_rates(cfg, a.prec)
    cpu = None
    if not a.no_cpu:
        log("cpu baseline: timing the oracle on a bounded sample (default threads, then one) ...")
        cpu = cpu_baseline_both(cfg, g["iterations"][-1])
        log(f"cpu baseline: projected {cpu['projected_s_per_solve']:.0f} s per solve "
            f"({cpu['cores']} threads), {cpu['one_thread']['projected_s_per_solve']:.0f} s "
            "on one thread")
    fflop = g["factor_flop"]
    ftf = fflop / (g["factor_ms"] * 1e-3) / 1e12
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
        "dtype": "f64" if a.prec == "fp64" else "f32-precond/f64-outer",
        "data": "synthetic plane-wave impedance data",
        "config": {"workload": cfg["name"], "k": cfg["k"], "n": cfg["n"], "p": cfg["p"],
                   "shift": str(cfg["s"]), "tol": cfg["tol"], "restart": cfg["restart"],
                   "nu": cfg["nu"], "omega": cfg["omega"], "precision": a.prec,
                   "iterations": g["iterations"]},
        "roofline": {"kernel": "multifrontal coarse solve (k_mf_sub for the bottom subtrees, "
                               "k_mf_solve per higher tree height and pass; unit: one coarse "
                               "system)", "bound": "hbm",
                     "achieved": cs_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": cs_gbs / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if (cfg["name"] == "p1_k400_n2048" and
                                                       a.prec == "fp64") else None,
                     "bytes_per_system": g["coarse_bytes"], "ms_per_system": g["coarse_ms"],
                     "systems": g["coarse_systems"],
                     "launches_per_system": g["launches_per_system"]},
        "setup_factor_ms": g["factor_ms"],
        "factorisation": {"kernel": "multifrontal factorisation (front assembly, extend-add, "
                                    "Gauss-Jordan and FP64 MFMA sweep inverses, complex GEMMs)",
                          "bound": "fp64", "ms": g["factor_ms"], "flop": fflop,
                          "achieved_tflops": ftf, "peak_tflops": FP64_MFMA_PEAK_TFLOPS,
                          "frac": ftf / FP64_MFMA_PEAK_TFLOPS},
        "stencil_passes": stencils,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    release()


def release():
    """Frees every device object before the interpreter exits (problems are closed by the
    steps; this drops torch's cached blocks once the device is idle)."""
    import gc
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def main_sweep(a, cfg):
    g = run_sweep(cfg, a.steps, a.warmup, a.prec)
    cs_gbs = g["coarse_bytes"] / (g["coarse_ms"] * 1e-3) / 1e9
    out = {
        "metric": "FGMRES solves/s",
        "value": g["solves"] / g["seconds"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * g["seconds"] / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.prec == "fp64" else "f32-precond/f64-outer",
        "data": "synthetic plane-wave impedance data",
        "config": {"workload": cfg["name"], "k": cfg["k"], "n": cfg["n"], "p": cfg["p"],
                   "shifts": len(g["betas"]), "angles": len(g["thetas"]), "tol": cfg["tol"],
                   "restart": cfg["restart"], "nu": cfg["nu"], "omega": cfg["omega"],
                   "precision": a.prec, "shifts_per_batch": g["group"]},
        "roofline": {"kernel": "multifrontal coarse solves, several shifts x right-hand sides "
                               "per launch (k_mf_solve; unit: one coarse system)",
                     "bound": "hbm", "achieved": cs_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": cs_gbs / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_system": g["coarse_bytes"], "ms_per_system": g["coarse_ms"],
                     "systems": g["coarse_systems"],
                     "launches_per_system": g["launches_per_system"]},
        "setup_factor_ms": g["factor_ms"],
        "sweep": {"beta_star": g["bstar"], "sigma_star": g["sigma"],
                  "mean_iterations_per_beta": [float(np.mean(x)) for x in g["its"]],
                  "betas": g["betas"], "converged": g["converged"],
                  "setup_s_per_sweep": g["setup_s"]},
        "cpu_baseline": None,
    }
    if not a.no_cpu:
        log("cpu baseline: timing the oracle on a bounded sample ...")
        its = float(np.mean(g["its"]))
        one = dict(cfg, s=1 + 1j * g["bstar"], theta=g["thetas"][0])
        cpu = cpu_baseline(one, int(round(its)))
        cpu["sample"] += f"; one solve at beta*={g['bstar']:.3f} with the sweep's mean iterations"
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
