"""Pins of the oracle's symmetric-sharing mode (Section 2.1, Notations: the
interaction matrix is taken symmetric; for a symmetric kernel the block of
the pair (C', C) is the transpose of the block of (C, C')).

Reading: in this mode only the block of each interaction-list pair whose
target box has the smaller index is compressed (by the same ACA as the
ordered build); its mirror is that block's exact transpose, so one factor
pair serves both orientations.

Pinned by: the operator the representation applies is exactly symmetric
(the ordered build's is not); the shared blocks are bit-identical to the
ordered build's; the product against the dense one (numpy/BLAS) at
tolerance 1e-10 and, at tolerance 0, to rounding; the per-row bound of the
ordered build; refusal of the non-symmetric test kernel."""
import numpy as np
import pytest

from paper_2204_05536_amd import inputs
from tests import npref

SPECS = {
    "log": {"kind": "log", "diag_mode": "replace", "diag_value": 1200.0},
    "mq": {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6},
    "gauss": {"kind": "gauss", "c": 0.05, "diag_mode": "add", "diag_value": 1e-4},
}


def _operator(H, n):
    """The matrix the representation applies, column by column (e_j products)."""
    A = np.empty((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        A[:, j] = H.matvec(e)
        e[j] = 0.0
    return A


@pytest.mark.parametrize("name", ["log", "mq"])
def test_applied_operator_is_exactly_symmetric(orc, name):
    rng = np.random.default_rng(31)
    n = 700
    xy = rng.uniform(-1, 1, (n, 2))
    Hs = orc.OracleH(xy, SPECS[name], 8, 1e-10, symmetric=True)
    assert Hs.symmetric and Hs.kappa >= 3
    As = _operator(Hs, n)
    assert np.array_equal(As, As.T)
    # the ordered build compresses both orientations apart: not symmetric
    Ho = orc.OracleH(xy, SPECS[name], 8, 1e-10)
    Ao = _operator(Ho, n)
    assert np.max(np.abs(Ao - Ao.T)) > 0.0
    # both approximate the same dense matrix
    K = npref.kernel_matrix(SPECS[name], xy)
    scale = np.max(np.abs(K - np.diag(np.diag(K))))
    assert np.max(np.abs(As - K)) <= 1e-8 * scale
    assert np.max(np.abs(Ao - K)) <= 1e-8 * scale


def test_shared_blocks_equal_the_ordered_build(orc):
    rng = np.random.default_rng(32)
    xy = rng.uniform(-1, 1, (3000, 2))
    spec = SPECS["mq"]
    Hs = orc.OracleH(xy, spec, 32, 1e-10, symmetric=True)
    Ho = orc.OracleH(xy, spec, 32, 1e-10)
    ts, to = Hs.il_table(), Ho.il_table()
    for f in ("level", "tgt", "src"):
        assert np.array_equal(ts[f], to[f])
    own = ts["tgt"] < ts["src"]
    assert np.array_equal(ts["kind"][own], to["kind"][own]) and np.array_equal(ts["rank"][own], to["rank"][own])
    key = {(int(l), int(t), int(s)): b for b, (l, t, s) in enumerate(zip(ts["level"], ts["tgt"], ts["src"]))}
    for b in np.nonzero(own)[0][::7]:
        ks, Us, Vs, Ds = Hs.il_factors(int(b))
        ko, Uo, Vo, Do = Ho.il_factors(int(b))
        assert ks == ko
        if ks == orc.BK_DENSE:
            assert np.array_equal(Ds, Do)
        else:
            assert np.array_equal(Us, Uo) and np.array_equal(Vs, Vo)
        # the mirror holds the transposed pair
        mb = key[(int(ts["level"][b]), int(ts["src"][b]), int(ts["tgt"][b]))]
        km, Um, Vm, Dm = Hs.il_factors(mb)
        assert km == ks and ts["rank"][mb] == ts["rank"][b]
        if km == orc.BK_DENSE:
            assert np.array_equal(Dm, Ds.T)
        else:
            assert np.array_equal(Um, Vs) and np.array_equal(Vm, Us)
    # ranks of the two orientations differ in the ordered build, not here
    mate = np.array([key[(int(l), int(s), int(t))] for l, t, s in zip(ts["level"], ts["tgt"], ts["src"])])
    assert np.array_equal(ts["rank"], ts["rank"][mate])
    assert not np.array_equal(to["rank"], to["rank"][mate])


@pytest.mark.parametrize("name", ["log", "mq", "gauss"])
def test_symmetric_product_vs_dense(orc, name):
    rng = np.random.default_rng(33)
    xy = rng.uniform(-1, 1, (2000, 2))
    x = rng.uniform(-1, 1, 2000)
    spec = SPECS[name]
    H = orc.OracleH(xy, spec, 32, 1e-10, symmetric=True)
    A = npref.kernel_matrix(spec, xy)
    assert np.linalg.norm(H.matvec(x) - A @ x) <= 1e-8 * np.linalg.norm(A @ x)


def test_symmetric_zero_tolerance_equals_dense(orc):
    rng = np.random.default_rng(34)
    xy = rng.uniform(-1, 1, (1500, 2)); x = rng.uniform(-1, 1, 1500)
    spec = {"kind": "log", "diag_mode": "replace", "diag_value": 1500.0}
    H = orc.OracleH(xy, spec, 16, 0.0, symmetric=True)
    assert np.all(H.il_table()["kind"] == 1)
    A = npref.kernel_matrix(spec, xy)
    assert np.linalg.norm(H.matvec(x) - A @ x) <= 1e-14 * np.linalg.norm(A @ x)


def test_symmetric_row_error_bound(orc):
    """Per-row error within 10 tol of sum_j |A_ij x_j|, as for the ordered build."""
    xy, b, kern, leaf, tol = inputs.workload("mq1m", n=16384)
    H = orc.OracleH(xy, kern, leaf, tol, symmetric=True)
    y = H.matvec(b)
    rows = np.random.default_rng(6).choice(16384, 64, replace=False)
    ye = orc.dense_rows(kern, xy, b, rows)
    absrow = np.array([np.sum(np.abs(orc.entries(kern, xy, np.full(16384, i), np.arange(16384)) * b)) for i in rows])
    assert np.max(np.abs(y[rows] - ye) / absrow) <= 10 * tol


def test_refusals(orc):
    rng = np.random.default_rng(35)
    xy = rng.uniform(-1, 1, (300, 2))
    with pytest.raises(orc.OracleError) as e:
        orc.OracleH(xy, {"kind": "sep", "c": 3, "diag_mode": "formula"}, 16, 1e-10, symmetric=True)
    assert e.value.code == orc.ORC_EINVAL
    with pytest.raises(orc.OracleError) as e:
        orc.OracleH(xy, SPECS["log"], 16, 1e-10, symmetric=True, adaptive=True)
    assert e.value.code == orc.ORC_EINVAL
