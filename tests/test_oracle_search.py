"""Pins of the golden-section shift search (Sec. 5) and of the sample draws."""

import math

import numpy as np
import pytest

from oracle import shiftsearch as O
from paper_2104_01439_amd import inputs


@pytest.mark.parametrize("xstar", [1.0, 1.13, 1.5, 1.87, 2.0])
def test_golden_section_finds_the_minimum_of_a_unimodal_function(xstar):
    f = lambda x: (x - xstar) ** 2
    x, trace = O.golden_section(f, 1.0, 2.0, 1e-2)
    assert abs(x - xstar) <= 1e-2
    # two initial points, then one new point per reduction of the bracket by the golden ratio
    n_red = math.ceil(math.log(1e-2) / math.log(O.GOLDEN))
    assert len(trace) == 2 + n_red
    # the inner points are the golden sections of the unit interval
    assert abs(trace[0][0] - (2 - O.GOLDEN)) < 1e-15 and abs(trace[1][0] - (1 + O.GOLDEN)) < 1e-15


def test_golden_section_brackets_shrink_by_the_golden_ratio():
    seen = []
    O.golden_section(lambda x: seen.append(x) or abs(x - 1.3), 1.0, 2.0, 1e-3)
    # consecutive new points on one side are golden sections of shrinking brackets:
    # all points stay inside [1, 2] and the last ones cluster at the minimum
    assert all(1.0 <= x <= 2.0 for x in seen)
    assert abs(seen[-1] - 1.3) < 5e-3


def test_golden_section_ties_move_the_lower_end():
    x, _ = O.golden_section(lambda x: 1.0, 1.0, 2.0, 1e-2)
    assert x > 2.0 - 1e-2


def test_shift_multiplier_gives_eps_k_to_sigma():
    for k, s in [(10.0, 1.0), (100.0, 1.5), (300.0, 2.0)]:
        m = O.shift_multiplier(k, s)
        assert m.real == 1.0 and abs(m.imag * k * k - k ** s) <= 1e-12 * k ** s


def test_objective_is_the_average_true_residual_reduction():
    """rho^end equals the true relative residual of the same solve."""
    from oracle import Problem
    s = inputs.shift_samples(1, seed=5, ells=(4,), orders=(1,))[0]
    F = inputs.sample_rhs(s)
    rho = O.objective(s["k"], s["n"], s["p"], 1.5, F)
    out = Problem(s["k"], s["n"], s["p"], O.shift_multiplier(s["k"], 1.5)).solve(F, tol=1e-8, m=50,
                                                                                maxit=50)
    its = out["iterations"]
    assert 0 < its <= 50
    assert abs(rho ** its - out["true_rel_res"]) <= 1e-12
    r = np.linalg.norm(F - Problem(s["k"], s["n"], s["p"], 1.0).A0 @ out["u"]) / np.linalg.norm(F)
    assert abs(r - out["true_rel_res"]) <= 1e-12


def test_sample_draws_follow_the_recipe():
    ss = inputs.shift_samples(300, seed=2)
    for s in ss:
        h = s["h"]
        assert s["p"] in (1, 2, 3) and 4 <= s["ell"] <= 10 and h == 2.0 ** -s["ell"]
        assert 3 * s["p"] / (16 * h) <= s["k"] <= 3 * s["p"] / (4 * h)
    assert {s["p"] for s in ss} == {1, 2, 3} and len({s["ell"] for s in ss}) == 7
    F = inputs.sample_rhs(ss[0])
    assert F.size == (ss[0]["p"] * ss[0]["n"] + 1) ** 2 and np.all(F.imag == 0)
    assert np.abs(F.real).max() <= 1 and np.array_equal(F, inputs.sample_rhs(ss[0]))
