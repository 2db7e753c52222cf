"""Pins of the oracle's adaptive-tree mode (the paper, end of Section 4:
the method carries over to an adaptive quadtree with small changes).

Reading: a box is split exactly when it holds more than N_max points;
blocks come from descending pairs of boxes from (root, root): two distinct
boxes whose closed squares share at most one point form one compressed
block, two leaves that share a segment (or the same leaf) one dense block,
any other pair is replaced by the pairs of their children.

Pinned by: the balanced tree it must reproduce exactly when the adaptive
rule stops every branch at one depth; the split rule checked box by box;
exact-once coverage of all N^2 point pairs by brute force; the block
geometry re-derived here from keys and levels; the zero-tolerance operator
against the dense product (numpy/BLAS); the per-row error bound at
tolerance 1e-10."""
import numpy as np
import pytest

from paper_2204_05536_amd import inputs

LOG = {"kind": "log", "diag_mode": "replace", "diag_value": 0.0}


def _mixture(n, seed):
    return inputs.gaussian_mixture(n, np.random.default_rng(seed), sigma=0.05)


def _square(level, key, R=1.0):
    """Closed square of box (level, key): integer corners on the 2^16 grid."""
    x = y = 0
    for b in range(level):
        d = (key >> (2 * b)) & 3
        x |= (d & 1) << b
        y |= (d >> 1) << b
    s = 1 << (16 - level)
    return x * s, (x + 1) * s, y * s, (y + 1) * s


def _common(a, b):
    """Lengths of the x and y overlaps of two closed squares (< 0: apart)."""
    return min(a[1], b[1]) - max(a[0], b[0]), min(a[3], b[3]) - max(a[2], b[2])


def _leaves(O):
    out = []
    for l in range(O.kappa + 1):
        L = O.level(l)
        has_child = np.zeros(len(L["key"]), bool)
        if l < O.kappa:
            has_child[O.level(l + 1)["parent"]] = True
        for b in np.nonzero(~has_child)[0]:
            out.append((l, int(b), int(L["begin"][b]), int(L["count"][b]), int(L["key"][b])))
    return out


def test_reproduces_the_balanced_tree(orc):
    """A 64 x 64 grid of cell centres with N_max = 20: every level-3 box holds
    64 points and every level-4 box 16, so the adaptive rule stops every
    branch at depth 4, the balanced tree's kappa.  Tree, block tables,
    factors and the product must be identical."""
    g = -1 + (np.arange(64) + 0.5) * (2 / 64)
    X, Y = np.meshgrid(g, g)
    xy = np.stack([X.ravel(), Y.ravel()], 1)
    xy = xy[np.random.default_rng(4).permutation(len(xy))]
    kern = dict(LOG, diag_value=4096.0)
    A = orc.OracleH(xy, kern, 20, 1e-10)
    B = orc.OracleH(xy, kern, 20, 1e-10, adaptive=True)
    assert B.adaptive and not A.adaptive
    assert A.kappa == B.kappa == 4
    assert np.array_equal(A.perm(), B.perm())
    for l in range(5):
        la, lb = A.level(l), B.level(l)
        for f in ("key", "begin", "count", "parent"):
            assert np.array_equal(la[f], lb[f]), (l, f)
    for x, y in zip(A.near_table(), B.near_table()):
        assert np.array_equal(x, y)
    ta, tb = A.il_table(), B.il_table()
    for f in ta:
        assert np.array_equal(ta[f], tb[f]), f
    _, _, itl, isl = B.block_levels()
    assert np.array_equal(itl, isl)
    x = np.random.default_rng(5).uniform(-1, 1, len(xy))
    assert np.array_equal(A.matvec(x), B.matvec(x))


def test_split_rule_and_leaf_order(orc):
    xy = _mixture(3000, 1)
    O = orc.OracleH(xy, LOG | {"diag_value": 3000.0}, 32, 1e-8, factors=False, adaptive=True)
    perm = O.perm()
    leaves = _leaves(O)
    levels = {l for l, *_ in leaves}
    assert len(levels) >= 3                      # leaves at several depths
    # every leaf holds at most N_max points; every box that was split more
    for l in range(O.kappa + 1):
        L = O.level(l)
        has_child = np.zeros(len(L["key"]), bool)
        if l < O.kappa:
            has_child[O.level(l + 1)["parent"]] = True
        assert np.all(L["count"][has_child] > 32)
        assert np.all(L["count"][~has_child] <= 32)
        assert np.all(L["count"] >= 1)
    # leaves tile [0, N) in Morton order of their squares; inside a leaf,
    # caller order; every point lies in its leaf's square
    leaves.sort(key=lambda t: t[2])
    assert leaves[0][2] == 0 and sum(c for *_, c, _ in leaves) == len(xy)
    for (l, b, b0, c, k), nxt in zip(leaves, leaves[1:] + [None]):
        if nxt is not None:
            assert nxt[2] == b0 + c
        idx = perm[b0:b0 + c]
        assert np.all(np.diff(idx) > 0)
        x0, x1, y0, y1 = (v / 2 ** 15 - 1 for v in _square(l, k))
        p = xy[idx]
        top = x1 == 1.0
        assert np.all((p[:, 0] >= x0) & ((p[:, 0] < x1) | (top & (p[:, 0] <= x1))))
        topy = y1 == 1.0
        assert np.all((p[:, 1] >= y0) & ((p[:, 1] < y1) | (topy & (p[:, 1] <= y1))))
    starts = [(_square(l, k)[0], _square(l, k)[2]) for l, b, b0, c, k in leaves]
    morton = [sum(((((sx >> i) & 1) | (((sy >> i) & 1) << 1)) << (2 * i)) for i in range(16)) for sx, sy in starts]
    assert morton == sorted(morton)


@pytest.mark.parametrize("seed,n,leaf", [(2, 600, 16), (3, 900, 24)])
def test_blocks_cover_every_pair_once_with_the_right_geometry(orc, seed, n, leaf):
    xy = _mixture(n, seed)
    O = orc.OracleH(xy, LOG | {"diag_value": float(n)}, leaf, 1e-8, factors=False, adaptive=True)
    perm = O.perm()
    levels = [O.level(l) for l in range(O.kappa + 1)]
    leafset = {(l, b) for l, b, *_ in _leaves(O)}
    ntl, nsl, itl, isl = O.block_levels()
    cover = np.zeros((n, n), np.int32)
    nt, ns = O.near_table()
    for tl, t, sl, s in zip(ntl, nt, nsl, ns):
        Lt, Ls = levels[tl], levels[sl]
        assert (tl, t) in leafset and (sl, s) in leafset
        wx, wy = _common(_square(tl, int(Lt["key"][t])), _square(sl, int(Ls["key"][s])))
        same = tl == sl and t == s
        assert same or (min(wx, wy) == 0 and max(wx, wy) > 0)      # the same leaf, or a shared segment
        r = perm[Lt["begin"][t]:Lt["begin"][t] + Lt["count"][t]]
        c = perm[Ls["begin"][s]:Ls["begin"][s] + Ls["count"][s]]
        cover[np.ix_(r, c)] += 1
    tab = O.il_table()
    for tl, t, sl, s in zip(itl, tab["tgt"], isl, tab["src"]):
        Lt, Ls = levels[tl], levels[sl]
        wx, wy = _common(_square(tl, int(Lt["key"][t])), _square(sl, int(Ls["key"][s])))
        assert wx < 0 or wy < 0 or (wx == 0 and wy == 0)           # at most one common point
        r = perm[Lt["begin"][t]:Lt["begin"][t] + Lt["count"][t]]
        c = perm[Ls["begin"][s]:Ls["begin"][s] + Ls["count"][s]]
        cover[np.ix_(r, c)] += 1
    assert np.all(cover == 1)
    assert np.any(itl != isl)     # blocks between boxes of different levels exist


def test_zero_tolerance_equals_dense_product(orc):
    xy = _mixture(700, 6)
    kern = {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}
    O = orc.OracleH(xy, kern, 20, 0.0, adaptive=True)
    x = np.random.default_rng(7).uniform(-1, 1, 700)
    A = orc.dense_matrix(kern, xy)
    y = O.matvec(x)
    yd = A @ x
    assert np.linalg.norm(y - yd) <= 1e-14 * np.linalg.norm(np.abs(A) @ np.abs(x))


@pytest.mark.parametrize("kern", [LOG | {"diag_value": 1500.0},
                                  {"kind": "gauss", "c": 0.05, "diag_mode": "add", "diag_value": 1e-4}])
def test_error_per_row_within_tolerance(orc, kern):
    xy = _mixture(1500, 8)
    O = orc.OracleH(xy, kern, 24, 1e-10, adaptive=True)
    x = np.random.default_rng(9).uniform(-1, 1, 1500)
    A = orc.dense_matrix(kern, xy)
    err = np.abs(O.matvec(x) - A @ x)
    scale = np.abs(A) @ np.abs(x)
    assert np.all(err <= 10 * 1e-10 * scale)


def test_adaptive_tree_on_clusters(orc):
    """On the 4-cluster Gaussian mixture the balanced tree goes as deep as
    the densest cluster everywhere; the adaptive tree stops each branch
    where it holds at most N_max points.  Its depth is still set by the
    densest cluster, but it has far fewer boxes and blocks (larger blocks),
    and stores about as many values at the same tolerance (the sparse
    regions hold few points either way)."""
    xy = _mixture(4000, 10)
    kern = {"kind": "gauss", "c": 0.05, "diag_mode": "add", "diag_value": 1e-4}
    B = orc.OracleH(xy, kern, 32, 1e-10)
    A = orc.OracleH(xy, kern, 32, 1e-10, adaptive=True)
    assert A.kappa <= B.kappa
    nb = lambda O: sum(len(O.level(l)["key"]) for l in range(O.kappa + 1))
    assert nb(A) < nb(B)

    def stored(O):
        tab = O.il_table()
        _, _, itl, isl = O.block_levels()
        tot = 0
        for q in range(len(tab["tgt"])):
            m = O.level(int(itl[q]))["count"][tab["tgt"][q]]
            n = O.level(int(isl[q]))["count"][tab["src"][q]]
            tot += m * n if tab["kind"][q] == 1 else tab["rank"][q] * (m + n)
        ntl, nsl, _, _ = O.block_levels()
        t, s = O.near_table()
        for q in range(len(t)):
            tot += O.level(int(ntl[q]))["count"][t[q]] * O.level(int(nsl[q]))["count"][s[q]]
        return tot
    assert len(A.il_table()["tgt"]) < 0.5 * len(B.il_table()["tgt"])
    assert stored(A) <= 1.02 * stored(B)
