"""Serving engine on the GPU: continuous batching gives each request exactly the result it
gets alone (same kernels, same order), admission respects the memory budget, errors are
reported per request."""

import math
import sys
import time

import numpy as np
import pytest

from oracle import Problem as OProblem

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


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


# (k, n, p, beta, theta): several classes, sizes and shifts, so that requests join and leave
# the running batch at different rounds
MIX = [
    (12.0, 16, 1, 0.4, 0.3), (25.0, 32, 2, 1.1, 2.0), (9.0, 8, 3, 0.7, 4.1),
    (30.0, 64, 1, 0.2, 5.5), (18.0, 16, 2, 0.9, 1.2), (40.0, 32, 3, 0.5, 0.8),
    (20.0, 64, 1, 1.4, 3.3), (14.0, 16, 3, 0.15, 2.6), (35.0, 64, 2, 0.6, 4.8),
]


def drain(eng, count, timeout_s=240):
    got = {}
    t0 = time.time()
    while len(got) < count:
        for d, u in eng.poll(wait_ms=500):
            got[d["id"]] = (d, u)
        assert time.time() - t0 < timeout_s, f"engine returned {len(got)} of {count}"
    return got


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_engine_results_equal_alone(hz, torch, prec):
    _log(f"[engine] {len(MIX)} requests, {prec}")
    eng = hz.Engine(max_active=4, setup_threads=2, tol=1e-10, prec=prec)
    for i, (k, n, p, b, th) in enumerate(MIX):
        eng.submit(i, k, 1.0 / n, p, 1 + 1j * b, theta=th)
    got = drain(eng, len(MIX))
    info = eng.info()
    # finished requests' memory is credited back once their frees have completed
    t0 = time.time()
    while info["bytes_in_use"] != 0 and time.time() - t0 < 30:
        time.sleep(0.05)
        info = eng.info()
    eng.close()
    assert info["completed"] == len(MIX) and info["admitted"] == 0 and info["bytes_in_use"] == 0
    for i, (k, n, p, b, th) in enumerate(MIX):
        d, u = got[i]
        assert d["status"] == 0 and d["converged"] == 1, d
        pr = hz.Problem(k, 1.0 / n, p, 1 + 1j * b, prec=prec)
        ua, ra = pr.solve(pr.planewave_rhs(th), tol=1e-10, history=False)
        assert ra["iterations"] == d["iterations"]
        assert torch.equal(ua, u), f"request {i} differs from its solve alone"
        assert d["latency_s"] >= d["queue_s"] >= 0


def test_engine_against_oracle(hz, torch):
    reqs = [(16.0, 24, 2, 0.5, 0.7), (22.0, 40, 1, 0.8, 2.2)]
    F0 = None
    eng = hz.Engine(max_active=2, tol=1e-10, prec="mixed")
    ops = []
    for i, (k, n, p, b, th) in enumerate(reqs):
        op = OProblem(k, n, p, 1 + 1j * b)
        F = op.planewave_rhs(th)
        ops.append((op, F))
        Fd = torch.from_numpy(F).cuda()
        torch.cuda.synchronize()          # the engine reads F on its own stream
        if i == 0:
            F0 = Fd                       # caller-provided right-hand side
            eng.submit(i, k, 1.0 / n, p, 1 + 1j * b, F=F0)
        else:
            eng.submit(i, k, 1.0 / n, p, 1 + 1j * b, theta=th)
    got = drain(eng, len(reqs))
    eng.close()
    for i, (op, F) in enumerate(ops):
        d, u = got[i]
        ro = op.solve(F, tol=1e-10)
        err = np.linalg.norm(u.cpu().numpy() - ro["u"]) / np.linalg.norm(ro["u"])
        _log(f"  request {i}: its {d['iterations']} oracle {ro['iterations']}, u rel err {err:.2e}")
        assert abs(d["iterations"] - ro["iterations"]) <= 1
        assert err <= 1e-8


def test_engine_admission_and_errors(hz, torch):
    small = 256 << 20
    eng = hz.Engine(hbm_budget=small, max_active=2, tol=1e-8)
    with pytest.raises(hz.HZError) as ei:
        eng.submit(0, 100.0, 1 / 256, 3, 1 + 0.5j, theta=0.1)     # needs GBs
    assert ei.value.status == hz.HZ_ENOMEM
    with pytest.raises(hz.HZError) as ei:
        eng.submit(1, 10.0, 1 / 15, 1, 1 + 0.5j, theta=0.1)       # odd n
    assert ei.value.status == hz.HZ_EINVAL
    with pytest.raises(hz.HZError):
        eng.submit(2, 10.0, 1 / 16, 1, 1 - 0.5j, theta=0.1)       # Im(s) < 0
    for i in range(6):
        eng.submit(10 + i, 10.0 + i, 1 / 32, 1 + i % 3, 1 + 0.5j, theta=0.2 * i)
    peak = 0
    t0 = time.time()
    got = {}
    while len(got) < 6:
        inf = eng.info()
        peak = max(peak, inf["admitted"])
        assert inf["bytes_in_use"] <= small
        for d, u in eng.poll(wait_ms=20):
            got[d["id"]] = d
        assert time.time() - t0 < 120
    assert peak <= 2
    assert all(d["status"] == 0 and d["converged"] == 1 for d in got.values())
    # destroying with queued work neither hangs nor reports dropped requests
    for i in range(4):
        eng.submit(100 + i, 20.0, 1 / 64, 2, 1 + 0.5j, theta=0.3)
    eng.close()


def test_mixed_setup_returns_its_temporaries():
    """A mixed-precision problem factors in FP64 into a stream-ordered temporary of the full
    FP64 factor size; after creation that memory is free again for anyone (the pool is
    trimmed), and destroying the problem returns the rest."""
    import torch
    from paper_2104_01439_amd import hz
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, _ = torch.cuda.mem_get_info()
    pr = hz.Problem(120.0, 1 / 256, 3, 1 + 0.5j, prec="mixed")     # FP64 factor 5.5 GB
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    held = pr.info()["footprint_bytes"]
    pr.close()
    torch.cuda.synchronize()
    free2, _ = torch.cuda.mem_get_info()
    print(f"held {held / 1e9:.2f} GB, free drop after create {(free0 - free1) / 1e9:.2f} GB, "
          f"after destroy {(free0 - free2) / 1e9:.2f} GB", flush=True)
    assert free0 - free1 <= held + (512 << 20)
    assert free0 - free2 <= 512 << 20
