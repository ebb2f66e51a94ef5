"""Right-preconditioned flexible GMRES(m) (Sec. 4, after Saad 1993).

Test infrastructure (see the package header).

Solves A_0 P^{-1} (P u) = F with a preconditioner that may change every step, keeping
the preconditioned directions Z. Orthogonalisation is classical Gram-Schmidt applied
twice (CGS2). The least-squares problem is reduced by complex Givens rotations.
Stopping follows the paper's rule on the residual of the unpreconditioned system,
relative to the initial residual ||F|| (zero initial guess): inside a cycle the
rotation estimate |g_{j+1}| is tested; at the end of a cycle the true residual
F - A_0 u is recomputed and must pass as well, else the method restarts, until the
total number of preconditioner applications reaches ``maxit``.
"""

import numpy as np


def givens(a, b):
    """Rotation (c real, s complex) with [c s; -conj(s) c] [a; b] = [r; 0]."""
    if a == 0:
        return 0.0, 1.0 + 0j
    r = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    return abs(a) / r, (a / abs(a)) * np.conj(b) / r


def fgmres(apply_A, precond, F, tol=1e-8, m=50, maxit=5000, record=False):
    """Returns dict(u, iterations, converged, hist, true_rel_res, rho[, cycles]).

    ``hist`` holds one relative residual estimate per iteration. With ``record`` the
    per-cycle bases (V, Z, Hbar) are returned for checking the Arnoldi relation.
    """
    F = np.asarray(F, complex)
    N = F.size
    normF = np.linalg.norm(F)
    u = np.zeros(N, complex)
    out = dict(u=u, iterations=0, converged=True, hist=[], true_rel_res=0.0, rho=0.0,
               cycles=[])
    if normF == 0.0:
        return out
    r = F.copy()
    beta = normF
    its = 0
    hist = []
    converged = False
    while True:
        V = np.zeros((m + 1, N), complex)
        Z = np.zeros((m, N), complex)
        H = np.zeros((m + 1, m), complex)
        cs = np.zeros(m)
        sn = np.zeros(m, complex)
        g = np.zeros(m + 1, complex)
        V[0] = r / beta
        g[0] = beta
        j_end = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = apply_A(Z[j])
            its += 1
            for _ in range(2):                      # CGS2
                hh = V[: j + 1].conj() @ w
                w = w - V[: j + 1].T @ hh
                H[: j + 1, j] += hh
            hnext = np.linalg.norm(w)
            H[j + 1, j] = hnext
            Hbar_col = H[: j + 2, j].copy()
            if hnext > 0:
                V[j + 1] = w / hnext
            for i in range(j):                      # previous rotations
                a, b = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * b
                H[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * b
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            a, b = H[j, j], H[j + 1, j]
            H[j, j] = cs[j] * a + sn[j] * b
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            est = abs(g[j + 1]) / normF
            hist.append(est)
            j_end = j + 1
            if record:
                out["cycles"].append(("col", j, Hbar_col))
            if est <= tol or its >= maxit or hnext == 0.0:
                break
        # y = H^{-1} g on the j_end x j_end upper triangle, u += Z y
        y = np.zeros(j_end, complex)
        for i in range(j_end - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1: j_end] @ y[i + 1: j_end]) / H[i, i]
        u = u + Z[:j_end].T @ y
        if record:
            out["cycles"].append(("basis", V[: j_end + 1].copy(), Z[:j_end].copy()))
        r = F - apply_A(u)
        beta = np.linalg.norm(r)
        true_rel = beta / normF
        if true_rel <= tol:
            converged = True
            break
        if its >= maxit:
            converged = False
            break
    out.update(u=u, iterations=its, converged=converged, hist=np.array(hist),
               true_rel_res=true_rel)
    out["rho"] = true_rel ** (1.0 / its) if its > 0 else 0.0
    return out
