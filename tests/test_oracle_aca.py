"""Pins for the oracle's adaptive cross approximation.

Against: a separable kernel of known exact rank (ACA must stop at that rank
and reproduce the block to rounding), LAPACK's SVD (error of the cross
approximation close to the tolerance, rank not below the epsilon-rank of the
paper's Section 2 definition), the prefix structure of ACA (pivots do not
depend on the tolerance), the zero-tolerance and storage rules, and the
multipole bound of the Section 3 lemma for one-box-away log blocks.
"""
import numpy as np
import pytest

from tests import npref

LOG = {"kind": "log", "diag_mode": "replace", "diag_value": 1.0}


def _boxes(rng, m, n, cx=(-0.75, -0.75), cy=(0.25, -0.75), side=0.5):
    X = np.array(cx) + rng.uniform(0, side, (m, 2))
    Y = np.array(cy) + rng.uniform(0, side, (n, 2))
    return np.concatenate([X, Y]), np.arange(m), np.arange(m, m + n)


@pytest.mark.parametrize("rank", [1, 3, 7])
def test_separable_kernel_exact_rank(orc, rank):
    rng = np.random.default_rng(rank)
    xy, rows, cols = _boxes(rng, 60, 50)
    spec = {"kind": "sep", "c": float(rank), "diag_mode": "formula"}
    kind, k, U, V, D = orc.aca(spec, xy, rows, cols, 1e-12)
    # the stopping test looks at the newest cross, so after the r exact
    # crosses one more step (of rounding-level size) may be taken
    assert kind == 0 and k in (rank, rank + 1)
    a1 = 1.3 * xy[rows, 0] + 0.7 * xy[rows, 1]
    b1 = 0.9 * xy[cols, 0] - 1.1 * xy[cols, 1]
    A = sum(np.outer(np.cos(q * a1), np.cos(q * b1)) for q in range(rank))
    nA = np.linalg.norm(A)
    assert np.linalg.norm(U[:, :rank] @ V[:, :rank].T - A) <= 1e-13 * nA
    assert np.linalg.norm(U @ V.T - A) <= 1e-13 * nA


@pytest.mark.parametrize("tol", [1e-4, 1e-8, 1e-12])
def test_vertex_block_error_near_tolerance(orc, tol):
    """Vertex-sharing boxes (Section 3): ACA error within 100 tol, rank at
    least the SVD epsilon-rank at tol / 10 is not required, but at least the
    epsilon-rank at 10 tol (ACA cannot beat the SVD)."""
    rng = np.random.default_rng(7)
    xy, rows, cols = _boxes(rng, 120, 110, cx=(-0.5, -0.5), cy=(0.0, 0.0))
    kind, k, U, V, D = orc.aca(LOG, xy, rows, cols, tol)
    A = npref.kernel_matrix(LOG, xy[rows], xy[cols], same=False)
    Ak = U @ V.T if kind == 0 else D
    err = np.linalg.norm(Ak - A) / np.linalg.norm(A)
    assert err <= 100 * tol
    s = np.linalg.svd(A, compute_uv=False)
    eps_rank = int(np.sum(s / s[0] > 10 * tol))
    assert k >= eps_rank


def test_prefix_property(orc):
    """Tolerance only truncates: factors at a loose tolerance are the leading
    columns of those at a tighter tolerance."""
    rng = np.random.default_rng(3)
    xy, rows, cols = _boxes(rng, 200, 180, cx=(-1.0, -1.0), cy=(0.0, -1.0), side=1.0)
    _, k1, U1, V1, _ = orc.aca(LOG, xy, rows, cols, 1e-4)
    _, k2, U2, V2, _ = orc.aca(LOG, xy, rows, cols, 1e-10)
    assert k1 < k2
    assert np.array_equal(U1, U2[:, :k1]) and np.array_equal(V1, V2[:, :k1])


def test_zero_tolerance_gives_exact_dense(orc):
    rng = np.random.default_rng(4)
    xy, rows, cols = _boxes(rng, 30, 25)
    kind, k, U, V, D = orc.aca(LOG, xy, rows, cols, 0.0)
    assert kind == 1 and k == 25
    # numpy's vectorised log may differ from libm's by an ulp
    assert np.allclose(D, npref.kernel_matrix(LOG, xy[rows], xy[cols], same=False), rtol=4e-16, atol=0)


def test_storage_rule_dense_when_factors_larger(orc):
    """k (m + n) >= m n: the dense block is smaller and exact, so it is kept."""
    rng = np.random.default_rng(5)
    xy, rows, cols = _boxes(rng, 12, 10, cx=(-0.5, -0.5), cy=(0.0, 0.0), side=0.5)
    kind, k, U, V, D = orc.aca(LOG, xy, rows, cols, 1e-10)
    assert kind == 1 and k * 22 >= 120
    assert np.allclose(D, npref.kernel_matrix(LOG, xy[rows], xy[cols], same=False), rtol=4e-16, atol=0)


def test_zero_block(orc):
    """A numerically zero block (far Gaussian) gives rank 0, not a crash."""
    xy = np.array([[-1.0, -1.0], [-0.99, -1.0], [1.0, 1.0], [0.99, 1.0]])
    g = {"kind": "gauss", "c": 0.01, "diag_mode": "add", "diag_value": 0.0}
    kind, k, U, V, D = orc.aca(g, xy, [0, 1], [2, 3], 1e-10)
    assert kind == 0 and k == 0


def test_multipole_rank_bound_one_box_away(orc):
    """Section 3 theorem, case (i): log interactions of boxes one box apart
    admit rank p + 1 with p = log(sqrt2 Q / ((3 - sqrt2) eps)) / log(3 / sqrt2)
    for absolute error eps.  With unit charges Q = n and eps = tol * |A|_max
    the ACA rank at relative tolerance tol stays within 1.5 (p + 1)."""
    rng = np.random.default_rng(8)
    side = 0.5
    n = 150
    X = np.array([-1.0, -0.25]) + rng.uniform(0, side, (n, 2))
    Y = np.array([0.0, -0.25]) + rng.uniform(0, side, (n, 2))  # one box away along x
    xy = np.concatenate([X, Y])
    for tol in (1e-6, 1e-10):
        _, k, _, _, _ = orc.aca(LOG, xy, np.arange(n), np.arange(n, 2 * n), tol)
        A = npref.kernel_matrix(LOG, X, Y, same=False)
        eps = tol * np.abs(A).max()
        p = np.log(np.sqrt(2) * n / ((3 - np.sqrt(2)) * eps)) / np.log(3 / np.sqrt(2))
        assert k <= 1.5 * (p + 1)
