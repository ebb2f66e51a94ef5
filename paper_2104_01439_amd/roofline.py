"""Algorithmic byte counts of the hot kernels (what the method must move, not what the
hardware moved) and the MI355X peaks they are set against."""

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published


def coarse_solve_bytes(n, p, itemsize=16, nrhs=1):
    """One coarse block triangular solve launch for nrhs right-hand sides: every stored
    block inverse read twice (forward and backward sweep; the last block only once), plus
    per right-hand side the coarse vector read and the solution written and re-read."""
    nc = n // 2
    Mc = p * nc + 1
    blocks = nc * (p * Mc) ** 2 + Mc ** 2
    bwd = blocks - Mc ** 2
    return (blocks + bwd) * itemsize + 3 * Mc * Mc * itemsize * nrhs


def factor_bytes(n, p, itemsize=16):
    """Stored coarse factor: nc blocks of (p Mc)^2 and one of Mc^2."""
    nc = n // 2
    Mc = p * nc + 1
    return (nc * (p * Mc) ** 2 + Mc ** 2) * itemsize


def stencil_apply_bytes(n, p, itemsize=16):
    """y = A x on the fine lattice: x read once, y written once."""
    M = p * n + 1
    return 2 * M * M * itemsize
