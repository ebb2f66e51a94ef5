"""Algorithmic byte counts of the hot kernels (what the method must move, not what the
hardware moved) and the MI355X peaks they are set against."""

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix, published

# Algorithmic bytes per fine dof of the fine-level passes (complex FP64 = 16 B; each operand
# counted once; a coarse vector is a quarter of a fine one):
#   A_0 apply        x read, y written                          32
#   first sweep      f read, u = omega D^-1 f written            32
#   Jacobi sweep     u, f read, u' written                       48
#   residual         u, f read, r written                        48
#   restriction      r read, r_c written (1/4)                   20
#   prolongation     e_c read (1/4), P e_c written               20
#   prolongation+add e_c read (1/4), u read, u + P e_c written   36
#   residual + restriction in one pass (P1): u, f read, r_c written (1/4)           36
#   sweep with the staged correction: u, f, e_c (1/4) read, u' written               52
STENCIL_BYTES_PER_DOF = {"a0_apply": 32, "jacobi_first": 32, "jacobi_sweep": 48,
                         "residual": 48, "restriction": 20, "prolongation": 20,
                         "prolongation_add": 36, "resid_restrict_fused": 36,
                         "sweep_staged_correction": 52}


# Per-point operators (heterogeneous k), P1: the 7 stored couplings of the point (16 B each)
# on top of the vectors of the constant-k pass, and the Jacobi multiplier per point.
STENCIL_PN_BYTES_PER_DOF_P1 = {"a0_apply": 7 * 16 + 32, "jacobi_sweep": 7 * 16 + 64,
                               "residual": 7 * 16 + 48}


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


def factor_flops(n, p):
    """Real flops of the coarse block factorisation: every block inverted by Gauss-Jordan,
    (p Mc)^3 complex multiply-adds (8 real flops each) per block."""
    nc = n // 2
    Mc = p * nc + 1
    return 8.0 * (nc * float(p * Mc) ** 3 + float(Mc) ** 3)
