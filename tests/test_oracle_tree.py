"""Pins for the oracle's box, quadtree, numbering and point order.

Each check compares the oracle against something fixed outside it: the
paper's numbering figure (Section 4, tests/golden/numbering_level2.txt), its
half-open split of B (Section 3), closed forms, or brute force in numpy.
"""
import os

import numpy as np
import pytest

from tests import npref

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_grid(name):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line)
    return rows


def test_paper_numbering_level2(orc):
    """Section 4 numbering figure, level 2: every printed id."""
    for ln in _read_grid("numbering_level2.txt"):
        ix, iy, pid = map(int, ln.split())
        assert orc.paper_id(ix, iy, 2) == pid


def test_paper_numbering_level1(orc):
    """Level-1 panel: 0 bottom-left, 1 bottom-right, 2 top-right, 3 top-left."""
    assert [orc.paper_id(0, 0, 1), orc.paper_id(1, 0, 1), orc.paper_id(1, 1, 1), orc.paper_id(0, 1, 1)] == [0, 1, 2, 3]


def test_paper_id_is_parent_times_four_plus_digit(orc):
    """The figure numbers children 4*parent + digit at every level."""
    for level in range(1, 5):
        for ix in range(2 ** level):
            for iy in range(2 ** level):
                pid = orc.paper_id(ix, iy, level)
                parent = orc.paper_id(ix // 2, iy // 2, level - 1) if level > 1 else 0
                assert pid // 4 == parent


def test_morton_key_matches_bit_interleave(orc):
    rng = np.random.default_rng(5)
    for level in (1, 3, 8, 16):
        ix = rng.integers(0, 2 ** level, 50); iy = rng.integers(0, 2 ** level, 50)
        ref = npref.morton_np(ix, iy, level)
        got = [orc.morton_key(int(a), int(b), level) for a, b in zip(ix, iy)]
        assert np.array_equal(np.array(got, np.uint64), ref)


@pytest.mark.parametrize("m,R", [(1.0, 1.0), (0.999, 1.0), (0.5, 0.5), (0.51, 1.0), (1.5, 2.0), (3e-3, 2.0 ** -8)])
def test_box_radius_smallest_power_of_two(orc, m, R):
    xy = np.array([[0.1 * m, -m], [0.0, 0.0]])
    assert orc.box_radius(xy) == R


def test_half_open_split_section3(orc):
    """Section 3 splits [-1,1]^2 into [-1,0) x [-1,1] and [0,1] x [-1,1]:
    x = 0 belongs to the right box, x = 1 to the right box, x = -1 to the left.
    Same rule on y.  With leaf_max = 1 and 4 points, one per cell, kappa = 1."""
    xy = np.array([[-1.0, -1.0], [0.0, -1.0], [1.0, 1.0], [-1.0, 0.0]])
    H = orc.OracleH(xy, {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 0.0}, leaf_max=1, factors=False)
    assert H.kappa == 1
    L = H.level(1)
    # Morton keys 0 (BL), 1 (BR), 3 (TR), 2 (TL): one point in each
    assert list(L["key"]) == [0, 1, 2, 3]
    perm = H.perm()
    # BL: point 0, BR: point 1, TL (key 2): point 3, TR (key 3): point 2
    assert list(perm) == [0, 1, 3, 2]


def test_kappa_rule_bruteforce(orc):
    """kappa = smallest depth with every box holding <= leaf_max points,
    counted in numpy by floor-based cells on dyadic-free random inputs."""
    rng = np.random.default_rng(11)
    for n, leaf in [(1, 1), (10, 3), (500, 16), (3000, 64), (4096, 64)]:
        xy = rng.uniform(-1, 1, (n, 2))
        H = orc.OracleH(xy, {"kind": "gauss", "c": 0.05, "diag_mode": "add", "diag_value": 1e-4},
                        leaf_max=leaf, factors=False)
        R = H.R
        for l in range(0, 20):
            cx = npref.cells_np(xy[:, 0], R, l); cy = npref.cells_np(xy[:, 1], R, l)
            _, counts = np.unique(cx * (2 ** l) + cy, return_counts=True)
            if counts.max() <= leaf:
                break
        assert H.kappa == l


def test_perm_on_dyadic_grid_is_morton_order(orc):
    """One point per cell centre of a 2^L x 2^L grid, fed in a shuffled
    order: the tree order is the Morton order of the cells."""
    L = 4
    s = 2 ** L
    ix, iy = np.meshgrid(np.arange(s), np.arange(s), indexing="ij")
    ix = ix.ravel(); iy = iy.ravel()
    centres = np.stack([-1 + (ix + 0.5) * 2 / s, -1 + (iy + 0.5) * 2 / s], axis=1)
    order = np.random.default_rng(3).permutation(s * s)
    xy = centres[order]
    H = orc.OracleH(xy, {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}, leaf_max=1, factors=False)
    assert H.kappa == L
    keys = npref.morton_np(ix[order], iy[order], L)
    assert np.array_equal(H.perm(), np.argsort(keys, kind="stable"))


def test_perm_ties_keep_caller_order(orc):
    """Points in the same leaf keep their caller order (stable order)."""
    rng = np.random.default_rng(4)
    xy = rng.uniform(-1, 1, (2000, 2))
    H = orc.OracleH(xy, {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}, leaf_max=40, factors=False)
    k = H.kappa
    cx = npref.cells_np(xy[:, 0], H.R, k); cy = npref.cells_np(xy[:, 1], H.R, k)
    keys = npref.morton_np(cx, cy, k)
    assert np.array_equal(H.perm(), np.lexsort((np.arange(2000), keys)))


def test_level_tables_consistent(orc):
    rng = np.random.default_rng(6)
    xy = rng.uniform(-1, 1, (3000, 2))
    H = orc.OracleH(xy, {"kind": "log", "diag_mode": "replace", "diag_value": 3000.0}, leaf_max=20, factors=False)
    k = H.kappa
    for l in range(k + 1):
        L = H.level(l)
        assert L["count"].sum() == 3000
        assert L["begin"][0] == 0
        assert np.array_equal(L["begin"][1:], np.cumsum(L["count"])[:-1])
        assert np.all(np.diff(L["key"].astype(np.int64)) > 0)
        if l > 0:
            P = H.level(l - 1)
            assert np.array_equal(P["key"][L["parent"]], L["key"] >> 2)
            # a parent's range covers its children
            assert np.all(P["begin"][L["parent"]] <= L["begin"])
    assert H.level(k)["count"].max() <= 20
    if k > 0:
        assert H.level(k - 1)["count"].max() > 20


def test_uniform_kappa_is_7_at_2_18(orc):
    """N = 2^18 uniform points, leaf 64: depth 7 (a level-6 box holds about
    64 points on average, so some exceed 64; a level-7 box about 16)."""
    from paper_2204_05536_amd import inputs
    xy, _, kern, leaf, _ = inputs.workload("mq1m", n=1 << 18)
    H = orc.OracleH(xy, kern, leaf, factors=False)
    assert H.kappa == 7
