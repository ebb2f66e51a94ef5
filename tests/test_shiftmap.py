"""The shift map of Sec. 5 (Table 1 weights) and its ADAM regression."""

import math

import numpy as np
import pytest

from paper_2104_01439_amd import shiftmap as M


@pytest.mark.parametrize("p", [1, 2, 3])
def test_map_structure(p):
    kc0, kc1, a0, a1 = M.TABLE1[p]
    for ell in (4, 6, 8, 10):
        kc = kc1 * math.exp(kc0 * ell)
        # beta(k_c) = 1: the map leaves sigma = 1 exactly at the critical wavenumber
        assert M.sigma_map(kc, ell, p) == pytest.approx(1.0, abs=1e-12)
        # below k_c the exponent is clamped to 1, far above it tends to 2
        assert M.sigma_map(0.5 * kc, ell, p) == 1.0
        assert M.sigma_map(kc + 50.0 / (a1 * math.exp(a0 * ell)), ell, p) == pytest.approx(2.0, abs=1e-12)
        ks = np.linspace(kc, 4 * kc, 50)
        s = M.sigma_map(ks, ell, p)
        assert np.all(np.diff(s) >= -1e-15) and s.min() >= 1.0 and s.max() <= 2.0


def test_map_value_one_e_folding_above_kc():
    # at k = k_c + 1/alpha: beta = 2 - e^-1
    kc0, kc1, a0, a1 = M.TABLE1[2]
    ell = 7
    k = kc1 * math.exp(kc0 * ell) + 1.0 / (a1 * math.exp(a0 * ell))
    assert M.sigma_map(k, ell, 2) == pytest.approx(2.0 - math.exp(-1.0), rel=1e-13)


def test_shift_from_map_gives_eps_k_to_sigma():
    for k, h, p in [(150.0, 1 / 512, 2), (900.0, 1 / 1024, 1), (40.0, 1 / 16, 3)]:
        sigma, s = M.shift_from_map(k, h, p)
        assert s.real == 1.0 and s.imag * k * k == pytest.approx(k ** sigma, rel=1e-13)
        assert sigma == M.sigma_map(k, math.log2(1 / h), p)


def test_sample_weights_count_order_and_level():
    ells = [4, 4, 5, 4, 6]
    ps = [1, 1, 1, 2, 1]
    w = M.sample_weights(ells, ps)
    assert np.allclose(w, [(5 / 2) ** 2, (5 / 2) ** 2, 25.0, 25.0, 25.0])


def test_fit_recovers_the_weights_of_noise_free_samples():
    """Samples drawn from the map with known weights (in the transition band, where the
    clamps are inactive) are fitted back from the paper's initial weights."""
    true = (0.45, 2.6, -0.6, 1.7)
    rng = np.random.default_rng(0)
    ell = rng.integers(4, 9, 400).astype(float)
    kc = true[1] * np.exp(true[0] * ell)
    alpha = true[3] * np.exp(true[2] * ell)
    k = kc + rng.uniform(0.05, 2.0, ell.size) / alpha
    sig = M.sigma_map(k, ell, weights=true)
    w = M.sample_weights(ell, np.ones_like(ell))
    init_loss = float(np.sum(w * (sig - M.sigma_map(k, ell, weights=(0.1, 1.0, -0.5, 1.0))) ** 2))
    est, loss = M.fit(k, ell, sig, w, epochs=20000, lr=1e-2)
    assert loss < 1e-4 * init_loss
    pred = M.sigma_map(k, ell, weights=est)
    assert np.abs(pred - sig).max() < 2e-2
