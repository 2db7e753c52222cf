"""h2d_matvec_noalloc: the single-RHS product on the library's fixed
per-GPU work array, called through the C ABI, against h2d_matvec (the
entry point that owns its work vectors) on the same handle and input.
Both run the same kernels in the same order, so the results must agree bit
for bit.  Two calls in a row, the second on a smaller handle, so the second
call runs on an array that still holds the first call's values."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2204_05536_amd import inputs
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


def _abi_noalloc(L, H, x, y, prec):
    strm = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.h2d_matvec_noalloc(H._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), prec, strm)


def _abi_matvec(L, H, x, y, prec):
    strm = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.h2d_matvec(H._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), 1, x.shape[0], prec, strm)


def test_noalloc_matches_matvec_twice_shrinking(orc):
    from paper_2204_05536_amd import hodlr2d
    L = hodlr2d.load()
    cases = [("mq1m", 1 << 16), ("log4096", 3000)]   # second call: a smaller input
    for name, n in cases:
        xy, b, kern, leaf, tol = inputs.workload(name, n=n)
        say(f"noalloc: {name} n={n}")
        H = hodlr2d.HODLR2D.build(dev(xy), kern, leaf, tol, precs=("fp16", "bf16"))
        x = dev(b)
        for prec in (0, 1, 2):
            y0 = torch.full_like(x, np.nan)
            y1 = torch.full_like(x, np.nan)
            assert _abi_matvec(L, H, x, y0, prec) == hodlr2d.H2D_OK
            assert _abi_noalloc(L, H, x, y1, prec) == hodlr2d.H2D_OK, L.h2d_last_error()
            a, c = host(y0), host(y1)
            assert np.all(np.isfinite(c))
            assert np.array_equal(a, c), (name, prec, np.max(np.abs(a - c)))
        # FP64 rows against the oracle's exact rows (the plain definition)
        rows = np.random.default_rng(1).choice(n, 16, replace=False)
        yd = orc.dense_rows(kern, xy, b, rows)
        err = np.max(np.abs(c_fp64(L, H, x)[rows] - yd)) / np.max(np.abs(yd))
        say(f"noalloc {name}: max row error vs exact rows {err:.2e}")
        assert err <= 1e-8
        H.close()


def c_fp64(L, H, x):
    y = torch.empty_like(x)
    assert _abi_noalloc(L, H, x, y, 0) == 0
    return host(y)


def test_noalloc_errors():
    from paper_2204_05536_amd import hodlr2d
    L = hodlr2d.load()
    xy, b, kern, leaf, tol = inputs.workload("log4096", n=500)
    H = hodlr2d.HODLR2D.build(dev(xy), kern, leaf, tol)
    x = dev(b); y = torch.empty_like(x)
    assert _abi_noalloc(L, H, x, y, 1) == hodlr2d.H2D_EUNSUPPORTED      # FP16 pool not built
    assert _abi_noalloc(L, H, x, y, 7) == hodlr2d.H2D_EINVAL
    strm = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.h2d_matvec_noalloc(H._h, None, C.c_void_p(y.data_ptr()), 0, strm) == hodlr2d.H2D_EINVAL
