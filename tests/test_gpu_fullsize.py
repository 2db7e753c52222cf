"""GPU parity at the benchmark's full size (N = 2^20, the configuration
bench.py times): structure bit-exact with the oracle, the FP64 product on
sampled rows against the oracle's exact O(N) rows, FP16/BF16 products
within their unit-roundoff bounds, and bitwise repeatability.

Row tolerance: for ACA tolerance tol the oracle's own rows stay within
10 tol of the exact product relative to sum_j |A_ij x_j| (pinned on the CPU
in test_oracle_matvec.py::test_row_error_bound)."""
import numpy as np
import pytest

from paper_2204_05536_amd import inputs
from tests import h2dfile
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

N = 1 << 20
U16 = 2.0 ** -11
UBF = 2.0 ** -8


@pytest.fixture(scope="module")
def mq_full(orc):
    from paper_2204_05536_amd import hodlr2d
    xy, b, kern, leaf, tol = inputs.workload("mq1m")
    assert xy.shape[0] == N
    say("full-size build", N)
    H = hodlr2d.HODLR2D.build(dev(xy), kern, leaf, tol, precs=("fp16", "bf16"))
    rows = np.sort(np.random.default_rng(77).choice(N, 48, replace=False))
    say("oracle exact rows")
    ye = orc.dense_rows(kern, xy, b, rows)
    absrow = np.array([np.sum(np.abs(orc.entries(kern, xy, np.full(N, i), np.arange(N)) * b)) for i in rows])
    return H, xy, b, kern, leaf, tol, rows, ye, absrow


def test_full_structure_bit_exact(orc, tmp_path, mq_full):
    H, xy, b, kern, leaf, tol, *_ = mq_full
    p = tmp_path / "s.h2dx"
    H.export(p, factors=False)
    F = h2dfile.read(p)
    say("oracle structure")
    O = orc.OracleH(xy, kern, leaf, tol, factors=False)
    assert F["kappa"] == O.kappa == 8
    assert np.array_equal(F["perm"], O.perm())
    for l in range(O.kappa + 1):
        L = O.level(l)
        for f in ("key", "begin", "count", "parent"):
            assert np.array_equal(F["levels"][l][f].astype(np.int64), L[f].astype(np.int64)), (l, f)
    t, s = O.near_table()
    assert np.array_equal(F["near_tgt"], t) and np.array_equal(F["near_src"], s)
    tab = O.il_table()
    assert np.array_equal(F["il_tgt"], tab["tgt"]) and np.array_equal(F["il_src"], tab["src"])
    assert np.array_equal(F["il_level"], tab["level"])


def test_full_fp64_rows_and_repeatability(mq_full):
    H, xy, b, kern, leaf, tol, rows, ye, absrow = mq_full
    x = dev(b)
    y1 = host(H.matvec(x)).copy()
    y2 = host(H.matvec(x))
    assert np.array_equal(y1, y2)
    err = np.abs(y1[rows] - ye) / absrow
    say("fp64 max row error", err.max())
    assert err.max() <= 10 * tol


@pytest.mark.parametrize("prec,u", [("fp16", U16), ("bf16", UBF)])
def test_full_half_precision_rows(mq_full, prec, u):
    """Stored values rounded to the half format (relative error <= u), FP32
    accumulation: each row within 4 u of sum_j |A_ij x_j| of the exact
    product (the factored low-rank parts can double the rounding)."""
    H, xy, b, kern, leaf, tol, rows, ye, absrow = mq_full
    y = host(H.matvec(dev(b), prec=prec))
    err = np.abs(y[rows] - ye) / absrow
    say(prec, "max row error / sum|A x|", err.max())
    assert err.max() <= 4 * u


def test_full_multi_rhs_rows(orc, mq_full):
    """The 16-RHS matrix-core product at N = 2^20, as bench.py times it:
    every right-hand side against the single-RHS product (rounding order
    only), and sampled rows of two right-hand sides against the oracle's
    exact rows."""
    H, xy, b, kern, leaf, tol, rows, ye, absrow = mq_full
    X = np.random.default_rng(7).uniform(-1, 1, (16, N))
    X[0] = b
    Y = host(H.matvec(dev(X)))
    for r in range(16):
        y1 = host(H.matvec(dev(X[r])))
        assert np.linalg.norm(Y[r] - y1) <= 1e-13 * np.linalg.norm(y1), r
    err = np.abs(Y[0][rows] - ye) / absrow
    assert err.max() <= 10 * tol
    r9 = rows[:12]
    ye9 = orc.dense_rows(kern, xy, X[9], r9)
    abs9 = np.array([np.sum(np.abs(orc.entries(kern, xy, np.full(N, i), np.arange(N)) * X[9])) for i in r9])
    err9 = np.abs(Y[9][r9] - ye9) / abs9
    say("16-RHS max row error", err.max(), err9.max())
    assert err9.max() <= 10 * tol


def test_batch_graph_full_sizes(orc):
    """The batched form on instances of the benchmark's recipe (the first 12
    of the 64: sizes log-uniform in [1e4, 5e5], disc / 4-cluster mixture,
    Gaussian kernel, 16 right-hand sides), tuned, captured and replayed:
    every replay equals the eager products, and sampled rows of each
    instance match the oracle's exact rows."""
    from paper_2204_05536_amd import hodlr2d
    import torch
    inst, kern, leaf, tol = inputs.batch_workload(64)
    inst = inst[:12]
    say("batch instances", [xy.shape[0] for xy, _ in inst])
    hs = [hodlr2d.HODLR2D.build(dev(xy), kern, leaf, tol) for xy, _ in inst]
    for H in hs:
        H.autotune(16)
    xs = [dev(X) for _, X in inst]
    ys = [torch.zeros_like(x) for x in xs]
    B = hodlr2d.Batch(hs, xs, ys)
    for rep in range(2):
        B.launch()
        torch.cuda.synchronize()
        for i, H in enumerate(hs):
            assert torch.equal(ys[i], H.matvec(xs[i])), (rep, i)
    rng = np.random.default_rng(3)
    worst = 0.0
    for i, (xy, X) in enumerate(inst):
        n = xy.shape[0]
        rows = np.sort(rng.choice(n, 4, replace=False))
        r = int(rng.integers(0, 16))
        ye = orc.dense_rows(kern, xy, X[r], rows)
        absr = np.array([np.sum(np.abs(orc.entries(kern, xy, np.full(n, j), np.arange(n)) * X[r])) for j in rows])
        err = np.abs(host(ys[i])[r][rows] - ye) / absr
        worst = max(worst, err.max())
    say("batch max row error / sum|A x|", worst)
    assert worst <= 10 * tol
    B.close()
