"""The shift search (Sec. 5) on the GPU against the oracle's: the objective of single
solves, and whole golden-section searches on small meshes."""

import sys

import numpy as np
import pytest

from oracle import shiftsearch as O
from paper_2104_01439_amd import inputs

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


SAMPLES = inputs.shift_samples(6, seed=11, ells=(4, 5))


def test_objective_matches_oracle(hz, torch):
    for s in SAMPLES[:3]:
        F = inputs.sample_rhs(s)
        for sigma in (1.0, 1.5, 2.0):
            pr = hz.Problem(s["k"], s["h"], s["p"], O.shift_multiplier(s["k"], sigma))
            u, r = pr.solve(torch.from_numpy(F).cuda(), tol=1e-8, maxit=50, restart=50,
                            history=False)
            rg = r["rel_res_true"] ** (1.0 / r["iterations"])
            ro = O.objective(s["k"], s["n"], s["p"], sigma, F)
            _log(f"  k={s['k']:.2f} ell={s['ell']} p={s['p']} sigma={sigma}: rho gpu {rg:.10f} "
                 f"oracle {ro:.10f} ({r['iterations']} its)")
            assert abs(rg - ro) <= 1e-8 * ro


def test_search_matches_oracle(hz, torch):
    Fs = [torch.from_numpy(inputs.sample_rhs(s)).cuda() for s in SAMPLES]
    res = hz.shift_search([(s["k"], s["h"], s["p"]) for s in SAMPLES], Fs)
    for s, r in zip(SAMPLES, res):
        so, trace = O.search(s["k"], s["n"], s["p"], inputs.sample_rhs(s))
        best = min(trace, key=lambda t: t[1])
        _log(f"  k={s['k']:.2f} ell={s['ell']} p={s['p']}: sigma gpu {r['sigma']:.6f} oracle "
             f"{so:.6f}, evaluations {r['evaluations']} / {len(trace)}, rho {r['rho']:.6f} / "
             f"{best[1]:.6f}")
        assert r["status"] == 0
        assert abs(r["sigma"] - so) <= 1e-2
        assert r["evaluations"] == len(trace)
        assert abs(r["rho"] - best[1]) <= 1e-8 * best[1]


def test_search_edge_cases(hz, torch):
    s = SAMPLES[0]
    F = torch.from_numpy(inputs.sample_rhs(s)).cuda()
    # a bracket already narrower than the tolerance: the two inner points only
    r = hz.shift_search([(s["k"], s["h"], s["p"])], [F], sigma_lo=1.4, sigma_hi=1.405, tol=1e-2)[0]
    assert r["evaluations"] == 2 and abs(r["sigma"] - 1.4025) < 1e-12
    # F = 0: every evaluation needs no iteration (rho = 0)
    Z = torch.zeros_like(F)
    r = hz.shift_search([(s["k"], s["h"], s["p"])], [Z])[0]
    assert r["rho"] == 0.0 and r["status"] == 0
    with pytest.raises(hz.HZError):
        hz.shift_search([(s["k"], 1 / 17, s["p"])], [F])
