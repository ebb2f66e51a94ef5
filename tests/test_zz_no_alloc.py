"""The allocation-free apply (hz_apply_noalloc) against hz_apply, through the C ABI.

Both run the same kernels with the same arithmetic, so every operator must agree bitwise;
the check is repeated on two calls in a row, the second on a smaller problem (the scratch
array keeps the first call's contents), and on a problem beyond the array's size, which
must be rejected.
"""

import sys

import numpy as np
import pytest

from paper_2104_01439_amd import inputs

pytestmark = pytest.mark.gpu

OPS = ["A0", "AEPS", "JACOBI", "RESTRICT", "PROLONG", "VCYCLE", "COARSE_SOLVE", "COARSE_A",
       "RESID_RESTRICT"]


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hz():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2104_01439_amd import hz as h
    h.lib()
    return h


def _inputs(torch, pr, op):
    coarse_in = op in ("PROLONG", "COARSE_SOLVE", "COARSE_A")
    n = pr.Nc if coarse_in else pr.N
    x = torch.from_numpy(inputs.random_complex(n, seed=31)).cuda()
    f = torch.from_numpy(inputs.random_complex(pr.N, seed=32)).cuda()
    return x, f


def _compare(hz, pr, prec):
    import torch
    for op in OPS:
        x, f = _inputs(torch, pr, op)
        ya = pr.apply(op, x, f, prec=prec)
        yb = pr.apply(op, x, f, prec=prec, noalloc=True)
        torch.cuda.synchronize()
        a, b = ya.cpu().numpy(), yb.cpu().numpy()
        e = np.linalg.norm(a - b) / max(np.linalg.norm(a), 1e-300)
        _log(f"  {prec} {op}: rel diff {e:.1e}, bitwise {torch.equal(ya, yb)}")
        assert np.isfinite(b).all()
        assert torch.equal(ya, yb), (op, prec, e)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_equals_apply_twice(hz, prec):
    # first a larger problem (several tiles, ragged), then a smaller one: the second call
    # runs on an array that still holds the first call's contents
    for (k, n, p) in [(45.0, 66, 3), (12.0, 18, 2)]:
        _log(f"[noalloc] k={k} n={n} p={p} {prec}")
        pr = hz.Problem(k, 1.0 / n, p, 1 + 0.5j, prec=prec)
        _compare(hz, pr, prec)
        pr.close()


def test_noalloc_rejects_beyond_maximum(hz):
    import torch
    pr = hz.Problem(50.0, 1.0 / 1024, 1, 1 + 0.5j, prec="mixed")   # 1.05 M fine dofs
    x = torch.zeros(pr.N, dtype=torch.complex128, device="cuda")
    with pytest.raises(hz.HZError) as ei:
        pr.apply("A0", x, prec="mixed", noalloc=True)
    assert ei.value.status == hz.HZ_EINVAL and "maximum" in str(ei.value)
    # an FP64 problem holds no FP32 factor until a mixed-precision call made one
    pr2 = hz.Problem(10.0, 1.0 / 16, 1, 1 + 0.5j)
    x2 = torch.zeros(pr2.N, dtype=torch.complex128, device="cuda")
    with pytest.raises(hz.HZError) as ei:
        pr2.apply("VCYCLE", x2, prec="mixed", noalloc=True)
    assert ei.value.status == hz.HZ_EINVAL
