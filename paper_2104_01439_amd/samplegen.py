"""Training data of the shift map (Sec. 5, data generation) on the GPU.

Every sample (k, ell, p) with its right-hand side (components uniform in [-1, 1], g = 0) is
searched for its near-optimal shift exponent by hz_shift_search (golden-section search on
[1, 2] to 1e-2; every objective evaluation is an FGMRES solve stopped at 1e-8 or after 50
iterations, run by the serving engine with the other samples' evaluations). The rows
(k, ell, p, sigma_hat, rho) are the data set D that shiftmap.fit() regresses.
"""

import torch

from . import hz, inputs


def generate(samples, prec="fp64", max_active=64, setup_threads=4):
    """Searches every sample (dicts from inputs.shift_samples); returns one row per sample."""
    Fs = [torch.from_numpy(inputs.sample_rhs(s)).to("cuda") for s in samples]
    res = hz.shift_search([(s["k"], s["h"], s["p"]) for s in samples], Fs, prec=prec,
                          max_active=max_active, setup_threads=setup_threads)
    return [dict(k=s["k"], ell=s["ell"], p=s["p"], sigma_hat=r["sigma"], rho=r["rho"],
                 sigma_best=r["sigma_best"], evaluations=r["evaluations"])
            for s, r in zip(samples, res)]
