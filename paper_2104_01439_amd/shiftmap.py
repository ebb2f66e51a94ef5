"""The near-optimal shift map of Sec. 5 and its regression.

For order p the map sends a wavenumber k and mesh level ell (h = 2^-ell) to the shift
exponent
    k_c(ell)     = kc1 exp(kc0 ell)
    alpha(ell)   = a1 exp(a0 ell)
    beta(k, ell) = 2 - exp(-alpha(ell) (k - k_c(ell)))
    sigma_p      = min(max(beta, 1), 2),
and the preconditioner's shift is eps = k^sigma (the multiplier s = 1 + i k^(sigma - 2) of
the k^2 mass term). TABLE1 holds the paper's weights (kc0, kc1, a0, a1) per order (Table 1;
they were fitted for Q_p elements, random f and g = 0).

fit() trains the four weights of one order on samples (k, ell, p, sigma_hat) by ADAM (Sec. 5:
learning rate 1e-3, initial weights (0.1, 1.0, -0.5, 1.0), 50 000 epochs) on the loss
    sum_i w_{ell_i, p}^-2 (sigma_hat_i - sigma_p(k_i, ell_i))^2,
w_{ell, p} = N_{ell, p} / |D| with N_{ell, p} the number of samples of order p AND level ell
(the printed definition omits the level condition, which would make the weight constant
within an order). Host-side (PyTorch on the CPU), like the paper's; not on the solve path.
"""

import math

import numpy as np

TABLE1 = {
    1: (0.4592788619853418, 2.5790032999702346, -0.6261637288068426, 1.7580549857142198),
    2: (0.5736926870738827, 2.5729974893966001, -0.6615199737374460, 1.5966386518185063),
    3: (0.6305770719029798, 2.4284320222555804, -0.4465407372367102, 0.1287828338493968),
}


def sigma_map(k, ell, p=None, weights=None):
    """sigma_p(k, ell) with the given weights (default: Table 1 for order p); k and ell may be
    arrays."""
    kc0, kc1, a0, a1 = weights if weights is not None else TABLE1[p]
    k = np.asarray(k, float)
    ell = np.asarray(ell, float)
    kc = kc1 * np.exp(kc0 * ell)
    alpha = a1 * np.exp(a0 * ell)
    beta = 2.0 - np.exp(-alpha * (k - kc))
    return np.minimum(np.maximum(beta, 1.0), 2.0)


def shift_from_map(k, h, p, weights=None):
    """(sigma, s): the map's exponent for wavenumber k, mesh size h (ell = log2(1/h)) and
    order p, and the preconditioner's shift multiplier s = 1 + i k^(sigma - 2)."""
    sigma = float(sigma_map(k, math.log2(1.0 / h), p, weights))
    return sigma, complex(1.0, k ** (sigma - 2.0))


def cell_shifts(k_cell, h, p, policy="map", weights=None):
    """Per-cell shift multipliers s_c = 1 + i eps_c / k_c^2 for a heterogeneous wavenumber
    (Sec. 6 compares eps in {k, k^(3/2), k^2, k^sigma_p} with k the local wavenumber):
    policy "k", "k1.5", "k2" (eps = k^e), or "map" (eps = k^sigma_p(k, ell), the map of Sec. 5
    evaluated at each cell's k, ell = log2(1/h))."""
    k = np.asarray(k_cell, float)
    if policy == "map":
        sigma = sigma_map(k, math.log2(1.0 / h), p, weights)
    else:
        sigma = {"k": 1.0, "k1.5": 1.5, "k2": 2.0}[policy]
    return 1.0 + 1j * k ** (sigma - 2.0)


def sample_weights(ells, ps):
    """w_{ell_i, p_i}^-2 per sample, w_{ell, p} = N_{ell, p} / |D|."""
    ells = np.asarray(ells)
    ps = np.asarray(ps)
    out = np.empty(len(ells))
    for i in range(len(ells)):
        nlp = np.count_nonzero((ps == ps[i]) & (ells == ells[i]))
        out[i] = (len(ells) / nlp) ** 2
    return out


def fit(k, ell, sigma_hat, weights, init=(0.1, 1.0, -0.5, 1.0), epochs=50000, lr=1e-3):
    """ADAM fit of (kc0, kc1, a0, a1) for one order; returns (weights, final loss)."""
    import torch

    kt = torch.tensor(np.asarray(k, float), dtype=torch.float64)
    lt = torch.tensor(np.asarray(ell, float), dtype=torch.float64)
    st = torch.tensor(np.asarray(sigma_hat, float), dtype=torch.float64)
    wt = torch.tensor(np.asarray(weights, float), dtype=torch.float64)
    th = torch.tensor(init, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([th], lr=lr)

    def loss_fn():
        kc = th[1] * torch.exp(th[0] * lt)
        alpha = th[3] * torch.exp(th[2] * lt)
        beta = 2.0 - torch.exp(-alpha * (kt - kc))
        sig = torch.clamp(beta, 1.0, 2.0)
        return torch.sum(wt * (st - sig) ** 2)

    for _ in range(epochs):
        opt.zero_grad()
        loss = loss_fn()
        loss.backward()
        opt.step()
    with torch.no_grad():
        final = float(loss_fn())
    return tuple(float(v) for v in th.detach()), final
