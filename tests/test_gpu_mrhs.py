"""Multi-RHS matvec (16 right-hand sides per pass on the matrix cores: FP64,
and FP32 for the FP16 / BF16 pools) against the single-RHS path and against
the oracle's Algorithm 2 on identical factors."""
import numpy as np
import pytest
import torch

from paper_2204_05536_amd import inputs
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2204_05536_amd import hodlr2d
    return hodlr2d


@pytest.mark.parametrize("nrhs", [2, 16, 21])
def test_multi_rhs_equals_single(nrhs):
    rng = np.random.default_rng(nrhs)
    xy = inputs.gaussian_mixture(6000, rng)
    spec = {"kind": "gauss", "c": 0.05, "diag_mode": "add", "diag_value": 1e-4}
    H = _lib().HODLR2D.build(dev(xy), spec, 32, 1e-10)
    X = rng.uniform(-1, 1, (nrhs, 6000))
    Y = host(H.matvec(dev(X)))
    for r in range(nrhs):
        y1 = host(H.matvec(dev(X[r])))
        assert np.linalg.norm(Y[r] - y1) <= 1e-13 * np.linalg.norm(y1), r


def test_multi_rhs_on_oracle_factors(orc, tmp_path):
    xy, b, kern, leaf, tol = inputs.workload("log4096")
    O = orc.OracleH(xy, kern, leaf, tol)
    p = tmp_path / "o.h2dx"
    O.export(p)
    H = _lib().HODLR2D.import_file(p)
    X = np.random.default_rng(4).uniform(-1, 1, (16, xy.shape[0]))
    Y = host(H.matvec(dev(X)))
    for r in range(16):
        yo = O.matvec(X[r])
        assert np.linalg.norm(Y[r] - yo) <= 1e-12 * np.linalg.norm(yo)


def test_multi_rhs_deep_tree_big_leaves():
    """Leaves above 64 points (two 64-row passes) and kappa >= 3."""
    rng = np.random.default_rng(9)
    xy = rng.uniform(-1, 1, (20000, 2))
    spec = {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}
    H = _lib().HODLR2D.build(dev(xy), spec, 100, 1e-10)
    X = rng.uniform(-1, 1, (16, 20000))
    Y = host(H.matvec(dev(X)))
    for r in (0, 7, 15):
        y1 = host(H.matvec(dev(X[r])))
        assert np.linalg.norm(Y[r] - y1) <= 1e-13 * np.linalg.norm(y1)


@pytest.mark.parametrize("nrhs", [1, 5, 16])
def test_leading_dimension_through_abi(nrhs):
    """Column-major X and Y with leading dimension ld > n, through the C ABI
    directly: the padding between columns is neither read into the result
    nor written."""
    import ctypes as C
    hd = _lib()
    rng = np.random.default_rng(31)
    n, ld = 5000, 5013
    xy = inputs.uniform_square(n, rng)
    spec = {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}
    H = hd.HODLR2D.build(dev(xy), spec, 64, 1e-10)
    Xp = rng.uniform(-1, 1, (nrhs, ld))
    Xp[:, n:] = np.nan   # padding must never be read
    Xd = dev(Xp)
    Yp = torch.full((nrhs, ld), 7.0, dtype=torch.float64, device="cuda")
    st = hd.load().h2d_matvec(H._h, C.c_void_p(Xd.data_ptr()), C.c_void_p(Yp.data_ptr()), nrhs, ld, 0,
                              C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    Y = host(Yp)
    assert np.all(Y[:, n:] == 7.0)
    for r in range(nrhs):
        y1 = host(H.matvec(dev(np.ascontiguousarray(Xp[r, :n]))))
        assert np.linalg.norm(Y[r, :n] - y1) <= 1e-13 * np.linalg.norm(y1), r


U16 = 2.0 ** -11   # unit roundoff of FP16
UBF = 2.0 ** -8    # unit roundoff of BF16


@pytest.mark.parametrize("prec,u", [("fp16", U16), ("bf16", UBF)])
@pytest.mark.parametrize("name", ["log4096", "mq5120_leaf100", "top_half_300"])
def test_half_multi_rhs_on_oracle_factors(orc, tmp_path, prec, u, name):
    """FP16 / BF16 pools made from the oracle's factors, 21 right-hand sides
    (a pass of 16 and a pass of 5): every row of every column within 4 u of
    sum_j |A_ij x_j| of the oracle's FP64 product (the bound of the
    single-RHS half path), and within FP32 rounding of the single-RHS half
    product of the same column (same stored values, FP32 sums in another
    order)."""
    from tests import npref
    if name == "log4096":
        xy, _, kern, leaf, tol = inputs.workload("log4096")
    elif name == "mq5120_leaf100":   # leaves of about 80 points: two 64-row passes per leaf
        xy = np.random.default_rng(12).uniform(-1, 1, (5120, 2))
        kern, leaf, tol = {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}, 100, 1e-10
    else:   # top half of B only: kappa = 2, empty walks above the leaves' parents
        g = np.random.default_rng(12)
        xy = np.stack([g.uniform(-1, 1, 300), g.uniform(0.01, 1, 300)], 1)
        kern, leaf, tol = {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}, 64, 1e-10
    n = xy.shape[0]
    O = orc.OracleH(xy, kern, leaf, tol)
    p = tmp_path / "o.h2dx"
    O.export(p)
    H = _lib().HODLR2D.import_file(p, precs=(prec,))
    X = np.random.default_rng(13).uniform(-1, 1, (21, n))
    Y = host(H.matvec(dev(X), prec=prec))
    Aabs = np.abs(npref.kernel_matrix(kern, xy))
    worst = 0.0
    for r in range(21):
        absrow = Aabs @ np.abs(X[r])
        yo = O.matvec(X[r])
        err = np.abs(Y[r] - yo) / absrow
        worst = max(worst, float(err.max()))
        assert np.all(np.isfinite(Y[r])) and err.max() <= 4 * u, (r, err.max())
        if r in (0, 15, 16, 20):
            y1 = host(H.matvec(dev(X[r]), prec=prec))
            assert np.max(np.abs(Y[r] - y1) / absrow) <= 1e-5, r
    say(f"{name} {prec} x21: max row error / sum|A x| = {worst:.2e} (4u = {4 * u:.1e})")
