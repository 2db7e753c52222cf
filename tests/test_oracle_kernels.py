"""Pins for the oracle's kernel entries against numpy closed forms.

Section 3 (log r), Section 5.1 (1/r with zero diagonal), Section 5.2
(phi_1, phi_2 with diagonal beta), and the multiquadric / Gaussian RBFs.
"""
import numpy as np
import pytest

from tests import npref

SPECS = [
    {"kind": "log", "diag_mode": "replace", "diag_value": 300.0},
    {"kind": "invr", "diag_mode": "replace", "diag_value": 0.0},
    {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6},
    {"kind": "gauss", "c": 0.05, "diag_mode": "add", "diag_value": 1e-4},
    {"kind": "phi1", "c": 1e-3, "diag_mode": "replace", "diag_value": 300.0},
    {"kind": "phi2", "c": 1e-3, "diag_mode": "replace", "diag_value": 300.0},
]


@pytest.mark.parametrize("spec", SPECS, ids=[s["kind"] for s in SPECS])
def test_kernel_matrix_matches_numpy(orc, spec):
    rng = np.random.default_rng(1)
    xy = rng.uniform(-1, 1, (300, 2))
    # a few pairs closer than a = 1e-3 exercise phi's inner branch
    xy[1] = xy[0] + [3e-4, -2e-4]
    xy[3] = xy[2] + [1e-5, 0.0]
    A = orc.dense_matrix(spec, xy)
    B = npref.kernel_matrix(spec, xy)
    assert np.allclose(A, B, rtol=1e-14, atol=1e-300)


def test_phi_branches_closed_form(orc):
    a = 1e-3
    xy = np.array([[0.0, 0.0], [0.5, 0.0], [a, 0.0], [a / 2, 0.0]])
    p1 = {"kind": "phi1", "c": a, "diag_mode": "replace", "diag_value": 4.0}
    p2 = {"kind": "phi2", "c": a, "diag_mode": "replace", "diag_value": 4.0}
    e = lambda s, i, j: orc.entries(s, xy, [i], [j])[0]
    assert e(p1, 0, 1) == pytest.approx(np.log(0.5) / np.log(a), rel=1e-15)
    assert e(p1, 0, 2) == pytest.approx(1.0, rel=1e-15)                     # r = a: log a / log a
    r = a / 2
    assert e(p1, 0, 3) == pytest.approx((r * np.log(r) - 1) / (a * np.log(a) - 1), rel=1e-15)
    assert e(p2, 0, 1) == pytest.approx(a / 0.5, rel=1e-15)
    assert e(p2, 0, 3) == pytest.approx(0.5, rel=1e-15)
    assert e(p1, 2, 2) == 4.0 and e(p2, 1, 1) == 4.0


def test_diagonal_by_index_not_distance(orc):
    """Two coincident points of the MQ kernel: off-diagonal gets phi(0) = 1,
    the diagonal gets 1 + shift."""
    xy = np.array([[0.25, 0.25], [0.25, 0.25]])
    s = {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}
    assert orc.entries(s, xy, [0, 0], [0, 1]).tolist() == [1.0 + 1e-6, 1.0]


def test_log_diagonal_replaced_by_n(orc):
    xy = np.random.default_rng(0).uniform(-1, 1, (64, 2))
    s = {"kind": "log", "diag_mode": "replace", "diag_value": 64.0}
    assert np.all(np.diag(orc.dense_matrix(s, xy)) == 64.0)
