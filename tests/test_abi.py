"""CPU checks of the C ABI: the library loads, exports every declared symbol, and its
host-only entry points (defaults, footprint model, argument validation) behave as declared.
No device work is launched here."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(hz_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def hz():
    from paper_2104_01439_amd import hz
    return hz


def test_library_exports_every_declared_symbol(hz):
    L = hz.lib()
    names = _declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
        assert n in hz._SIGS, f"binding lacks {n}"


def test_default_options(hz):
    o = hz.options()
    assert (o.nu, o.omega, o.restart, o.maxit, o.tol, o.prec) == (2, 0.6, 50, 5000, 1e-8, 0)


def test_footprint_model(hz):
    # invalid parameters give 0
    assert hz.footprint_estimate(10.0, 1 / 63, 1) == 0
    assert hz.footprint_estimate(10.0, 1 / 64, 4) == 0
    assert hz.footprint_estimate(-1.0, 1 / 64, 1) == 0
    # FP64 P1 n=2048: Krylov basis and preconditioned vectors, (51 + 50) fine vectors, plus
    # the multifrontal coarse factor (about 1.2e8 complex entries, 16 B each: far below the
    # 1025 x 1025 x 1025 x 16 B = 17.2 GB of dense block inverses of the block-tridiagonal
    # factor)
    fp = hz.footprint_estimate(400.0, 1 / 2048, 1, prec="fp64")
    krylov = (51 + 50) * 2049 ** 2 * 16
    assert krylov + 1.5e9 < fp < krylov + 3.5e9
    fm = hz.footprint_estimate(400.0, 1 / 2048, 1, prec="mixed")
    assert fm < fp
    # grows with n and p
    assert hz.footprint_estimate(50.0, 1 / 64, 1) < hz.footprint_estimate(50.0, 1 / 128, 1)
    assert hz.footprint_estimate(50.0, 1 / 64, 1) < hz.footprint_estimate(50.0, 1 / 64, 3)


def test_batch_workspace_model(hz):
    assert hz.batch_workspace_bytes(1 / 63, 1, 2, 4) == 0
    assert hz.batch_workspace_bytes(1 / 64, 1, 0, 4) == 0
    # P2 n=512: per solve V (51) + Z (50) + r, w, F, u, V-cycle scratch (3 fine, 2 coarse
    # vectors) and the coarse solve's work (the multifrontal update vectors: between one and
    # four coarse vectors), FP64
    N, Nc = 1025 ** 2, 513 ** 2
    b = hz.batch_workspace_bytes(1 / 512, 2, 8, 4, prec="fp64")
    per = (51 + 50 + 4 + 3) * N * 16 + 2 * Nc * 16
    assert 32 * (per + Nc * 16) <= b < 32 * (per + 4 * Nc * 16) + 1e8
    assert hz.batch_workspace_bytes(1 / 512, 2, 8, 4, prec="mixed") < b
    assert hz.batch_workspace_bytes(1 / 512, 2, 8, 4) > hz.batch_workspace_bytes(1 / 512, 2, 4, 4)


@pytest.mark.parametrize("k,h,p,s", [
    (10.0, 1 / 63, 1, 1 + 0.5j),      # odd n
    (10.0, 1 / 64, 4, 1 + 0.5j),      # bad order
    (10.0, 1 / 64, 1, 1 + 0.0j),      # no imaginary shift: the unpivoted coarse LU needs Im(s) > 0
    (10.0, 1 / 64, 1, 1 - 0.5j),
    (0.0, 1 / 64, 1, 1 + 0.5j),
    (float("nan"), 1 / 64, 1, 1 + 0.5j),
    (10.0, 1 / 8192, 1, 1 + 0.5j),    # beyond the supported size
])
def test_create_rejects_invalid_parameters(hz, k, h, p, s):
    handle = ctypes.c_void_p()
    o = hz.options()
    st = hz.lib().hz_create_problem(k, h, p, hz.C64(s.real, s.imag), ctypes.byref(o), None,
                                    ctypes.byref(handle))
    assert st == hz.HZ_EINVAL
    assert handle.value is None
    assert len(hz.lib().hz_last_error()) > 0


@pytest.mark.parametrize("field,val", [("restart", 0), ("restart", 65), ("nu", -1), ("omega", 0.0),
                                       ("omega", 2.5), ("maxit", 0), ("tol", -1.0), ("prec", 7)])
def test_create_rejects_invalid_options(hz, field, val):
    handle = ctypes.c_void_p()
    o = hz.options()
    setattr(o, field, val)
    st = hz.lib().hz_create_problem(10.0, 1 / 64, 1, hz.C64(1, 0.5), ctypes.byref(o), None,
                                    ctypes.byref(handle))
    assert st == hz.HZ_EINVAL


def test_null_arguments(hz):
    L = hz.lib()
    assert L.hz_solve(None, None, None, None, None, None, None) == hz.HZ_EINVAL
    assert L.hz_apply(None, 0, None, None, None, 0, None) == hz.HZ_EINVAL
    assert L.hz_apply_noalloc(None, 0, None, None, None, 0, None) == hz.HZ_EINVAL
    assert L.hz_problem_info(None, None, None, None) == hz.HZ_EINVAL
    L.hz_destroy_problem(None)


@pytest.mark.parametrize("bad", ["k_zero", "k_nan", "s_real", "s_neg", "odd_n", "null"])
def test_create_cells_rejects_invalid_cells(hz, bad):
    """Per-cell k and shift are validated on the host, naming the first bad cell."""
    import numpy as np
    n = 8 if bad != "odd_n" else 7
    kc = np.full((n, n), 5.0)
    sc = np.full((n, n), 1 + 0.5j)
    if bad == "k_zero":
        kc[3, 2] = 0.0
    elif bad == "k_nan":
        kc[0, 7] = float("nan")
    elif bad == "s_real":
        sc[5, 5] = 1.0
    elif bad == "s_neg":
        sc[1, 0] = 1 - 0.2j
    handle = ctypes.c_void_p()
    o = hz.options()
    args = (None, None) if bad == "null" else (kc.ctypes.data, sc.ctypes.data)
    st = hz.lib().hz_create_problem_cells(*args, 1.0 / n, 1, ctypes.byref(o), None,
                                          ctypes.byref(handle))
    assert st == hz.HZ_EINVAL and handle.value is None
    msg = hz.lib().hz_last_error().decode()
    if bad == "k_zero":
        assert "k_cell[26]" in msg
    if bad == "s_real":
        assert "s_cell[45]" in msg


def test_gaussian_rhs_rejects_null(hz):
    L = hz.lib()
    assert L.hz_gaussian_rhs(None, 0.5, 0.5, 2.0, 1000.0, None, None) == hz.HZ_EINVAL


def test_inputs_are_seeded():
    from paper_2104_01439_amd import inputs
    a = inputs.random_complex(100, seed=3)
    b = inputs.random_complex(100, seed=3)
    assert (a == b).all() and abs(a.real).max() <= 1
    th = inputs.sweep_thetas()
    assert len(th) == 4 and all(0 <= t < 6.2832 for t in th)
    betas = inputs.sweep_betas()
    assert len(betas) == 64 and betas[0] == 0.05 and abs(betas[-1] - 1.5) < 1e-15
    reqs = inputs.serving_requests(200, seed=1)
    assert all(r["k"] / (r["n"] * r["p"]) <= 0.3 for r in reqs)
    assert all(r["n"] // 2 * 2 == r["n"] for r in reqs)
