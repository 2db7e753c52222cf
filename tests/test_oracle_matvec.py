"""Pins for the oracle's Algorithm 2 (matvec) and restarted GMRES.

Against: the dense O(N^2) product built by numpy from the kernel formulas
(BLAS dgemv), the zero-tolerance build (every block exact, so the product
equals the dense one to rounding), error decreasing with the ACA tolerance,
and LAPACK's direct solve.
"""
import numpy as np
import pytest

from paper_2204_05536_amd import inputs
from tests import npref


def _offdiag_rel(y, A, x):
    Aoff = A - np.diag(np.diag(A))
    return np.linalg.norm(y - A @ x) / np.linalg.norm(Aoff @ x)


def test_log4096_matvec_vs_dense(orc):
    """N = 4096 uniform, log kernel with diagonal N, leaf 64, tol 1e-10:
    the error relative to the off-diagonal product stays within 10 tol."""
    xy, b, kern, leaf, tol = inputs.workload("log4096")
    H = orc.OracleH(xy, kern, leaf, tol)
    A = npref.kernel_matrix(kern, xy)
    y = H.matvec(b)
    assert H.kappa == 4
    assert _offdiag_rel(y, A, b) <= 10 * tol


@pytest.mark.parametrize("spec", [
    {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6},
    {"kind": "gauss", "c": 0.05, "diag_mode": "add", "diag_value": 1e-4},
    {"kind": "invr", "diag_mode": "replace", "diag_value": 0.0},
    {"kind": "phi1", "c": 1e-3, "diag_mode": "replace", "diag_value": 2000.0},
    {"kind": "phi2", "c": 1e-3, "diag_mode": "replace", "diag_value": 2000.0},
], ids=["mq", "gauss", "invr", "phi1", "phi2"])
def test_kernels_matvec_vs_dense(orc, spec):
    rng = np.random.default_rng(21)
    xy = rng.uniform(-1, 1, (2000, 2))
    x = rng.uniform(-1, 1, 2000)
    H = orc.OracleH(xy, spec, 32, 1e-10)
    A = npref.kernel_matrix(spec, xy)
    assert np.linalg.norm(H.matvec(x) - A @ x) <= 1e-8 * np.linalg.norm(A @ x)


def test_zero_tolerance_equals_dense(orc):
    rng = np.random.default_rng(22)
    xy = rng.uniform(-1, 1, (1500, 2)); x = rng.uniform(-1, 1, 1500)
    spec = {"kind": "log", "diag_mode": "replace", "diag_value": 1500.0}
    H = orc.OracleH(xy, spec, 16, 0.0)
    tab = H.il_table()
    assert np.all(tab["kind"] == 1)
    A = npref.kernel_matrix(spec, xy)
    assert np.linalg.norm(H.matvec(x) - A @ x) <= 1e-14 * np.linalg.norm(A @ x)


def test_error_decreases_with_tolerance(orc):
    rng = np.random.default_rng(23)
    xy = rng.uniform(-1, 1, (2500, 2)); x = rng.uniform(-1, 1, 2500)
    spec = {"kind": "log", "diag_mode": "replace", "diag_value": 2500.0}
    A = npref.kernel_matrix(spec, xy)
    errs = []
    for tol in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10, 1e-12):
        H = orc.OracleH(xy, spec, 32, tol)
        errs.append(_offdiag_rel(H.matvec(x), A, x))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-10


def test_single_leaf_is_dense(orc):
    """N <= leaf_max: kappa = 0, the root is the only leaf, one dense block."""
    rng = np.random.default_rng(24)
    xy = rng.uniform(-1, 1, (40, 2)); x = rng.uniform(-1, 1, 40)
    spec = {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}
    H = orc.OracleH(xy, spec, 64, 1e-10)
    assert H.kappa == 0 and len(H.il_table()["level"]) == 0
    A = npref.kernel_matrix(spec, xy)
    assert np.allclose(H.matvec(x), A @ x, rtol=1e-14, atol=1e-14)


def test_duplicate_points_rejected_for_singular_kernels(orc):
    xy = np.array([[0.1, 0.2], [0.5, 0.5], [0.1, 0.2]])
    with pytest.raises(orc.OracleError) as e:
        orc.OracleH(xy, {"kind": "log", "diag_mode": "replace", "diag_value": 3.0}, 8, 1e-10)
    assert e.value.code == orc.ORC_EDUP
    orc.OracleH(xy, {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}, 8, 1e-10)


def test_gmres_vs_lapack(orc):
    """log + N at N = 4096 is well conditioned: GMRES(50) reaches 1e-8 in a
    handful of iterations and matches the direct solve to cond * tol."""
    xy, b, kern, leaf, tol = inputs.workload("log4096")
    H = orc.OracleH(xy, kern, leaf, tol)
    x, it, rr, st = H.gmres(b, 1e-8, 50, 500)
    assert st == 0 and rr <= 1e-8 and it <= 12
    A = npref.kernel_matrix(kern, xy)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 1e-7
    # the residual the oracle reports is the true HODLR2D residual
    assert np.linalg.norm(b - H.matvec(x)) / np.linalg.norm(b) == pytest.approx(rr, rel=1e-6)


def test_gmres_restart_and_cap(orc):
    """An ill-conditioned system (MQ + 1e-6 I) with a tiny cap ends with the
    non-convergence status and the true residual of the iterate returned."""
    rng = np.random.default_rng(25)
    xy = rng.uniform(-1, 1, (600, 2)); b = rng.uniform(-1, 1, 600)
    spec = {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}
    H = orc.OracleH(xy, spec, 32, 1e-10)
    x, it, rr, st = H.gmres(b, 1e-12, 5, 12)
    assert st == orc.ORC_ENOCONV and it == 12
    assert np.linalg.norm(b - H.matvec(x)) / np.linalg.norm(b) == pytest.approx(rr, rel=1e-9)


def test_row_error_bound(orc):
    """Per-row error of Algorithm 2 stays within 10 tol of the exact row,
    relative to sum_j |A_ij x_j| (the bound the GPU full-size test uses)."""
    for name in ("mq1m", "log1m"):
        xy, b, kern, leaf, tol = inputs.workload(name, n=16384)
        H = orc.OracleH(xy, kern, leaf, tol)
        y = H.matvec(b)
        rows = np.random.default_rng(5).choice(16384, 64, replace=False)
        ye = orc.dense_rows(kern, xy, b, rows)
        absrow = np.array([np.sum(np.abs(orc.entries(kern, xy, np.full(16384, i), np.arange(16384)) * b)) for i in rows])
        assert np.max(np.abs(y[rows] - ye) / absrow) <= 10 * tol
