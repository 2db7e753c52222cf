"""One factor pair per interaction-list pair on the GPU (build flag
H2D_BUILD_SYMMETRIC) against the oracle's symmetric mode: the product on
the oracle's own factors (imported from its ordered file, whose mirror
blocks are exact transposes) within 1e-12, with bitwise repeatability; the
GPU-built operator within the ACA tolerance of the dense product (and equal
to it at tolerance 0) while storing about half the ordered form's values;
the export round trip; plain GMRES against the oracle's solution; the
refusals; and the full-size product on sampled rows against the oracle's
exact O(N) rows."""
import numpy as np
import pytest

from paper_2204_05536_amd import inputs
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

LOG = {"kind": "log", "diag_mode": "replace"}
MQ = {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}
GAUSS = {"kind": "gauss", "c": 0.05, "diag_mode": "add", "diag_value": 1e-4}
INVR = {"kind": "invr", "diag_mode": "replace", "diag_value": 0.0}
PHI1 = {"kind": "phi1", "c": 1e-3, "diag_mode": "replace", "diag_value": 2000.0}


def _lib():
    from paper_2204_05536_amd import hodlr2d
    return hodlr2d


def _grid():
    g = -1 + (np.arange(64) + 0.5) * (2 / 64)
    X, Y = np.meshgrid(g, g)
    xy = np.stack([X.ravel(), Y.ravel()], 1)
    return xy[np.random.default_rng(4).permutation(len(xy))]


def _case(name):
    r = np.random.default_rng
    if name == "log4096":
        xy, _, kern, leaf, _ = inputs.workload("log4096")
        return xy, kern, leaf
    if name == "mq6000_leaf32":
        return r(1).uniform(-1, 1, (6000, 2)), MQ, 32
    if name == "gauss5000_leaf16":
        return r(2).uniform(-1, 1, (5000, 2)), GAUSS, 16
    if name == "invr3000_leaf8":
        return r(3).uniform(-1, 1, (3000, 2)), INVR, 8
    if name == "phi1_2500_leaf20":
        return r(5).uniform(-1, 1, (2500, 2)), PHI1, 20
    if name == "mixture6000_log":
        return inputs.gaussian_mixture(6000, r(6)), LOG | {"diag_value": 6000.0}, 40
    if name == "grid_log":
        return _grid(), LOG | {"diag_value": 4096.0}, 20
    if name == "kappa1":
        return r(7).uniform(-1, 1, (120, 2)), MQ, 64
    if name == "kappa0":
        return r(8).uniform(-1, 1, (50, 2)), MQ, 64
    raise ValueError(name)


CASES = ["log4096", "mq6000_leaf32", "gauss5000_leaf16", "invr3000_leaf8", "phi1_2500_leaf20", "mixture6000_log",
         "grid_log", "kappa1", "kappa0"]


@pytest.mark.parametrize("name", CASES)
def test_matvec_on_oracle_factors(orc, tmp_path, name):
    xy, kern, leaf = _case(name)
    say(f"symmetric, oracle factors: {name} n={len(xy)} leaf={leaf}")
    O = orc.OracleH(xy, kern, leaf, 1e-10, symmetric=True)
    p = tmp_path / "o.h2dx"
    O.export(p)
    H = _lib().HODLR2D.import_file(p, symmetric=True)
    I = H.info()
    assert I["n_il"] == len(O.il_table()["tgt"]) and I["kappa"] == O.kappa
    x = np.random.default_rng(3).uniform(-1, 1, len(xy))
    yo = O.matvec(x)
    yg = host(H.matvec(dev(x))).copy()
    e = yg - yo
    say(f"{name}: kappa {O.kappa}, |y_gpu - y_oracle| / |y_oracle| = {np.linalg.norm(e) / np.linalg.norm(yo):.2e}")
    assert np.linalg.norm(e) <= 1e-12 * np.linalg.norm(yo)
    assert np.max(np.abs(e)) <= 1e-12 * np.max(np.abs(yo))
    assert np.array_equal(host(H.matvec(dev(x))), yg)
    # several right-hand sides: one at a time
    X = np.random.default_rng(9).uniform(-1, 1, (2, len(xy)))
    Y = host(H.matvec(dev(X)))
    for r in range(2):
        assert np.array_equal(Y[r], host(H.matvec(dev(X[r]))))


def test_import_refuses_an_ordered_file(orc, tmp_path):
    """The ordered build compresses both orientations apart: its mirrors are
    not transposes, so sharing them is refused."""
    xy, kern, leaf = _case("mq6000_leaf32")
    O = orc.OracleH(xy, kern, leaf, 1e-10)
    p = tmp_path / "o.h2dx"
    O.export(p)
    h = _lib()
    with pytest.raises(h.H2DError) as e:
        h.HODLR2D.import_file(p, symmetric=True)
    assert e.value.code == h.H2D_EINVAL
    h.HODLR2D.import_file(p)   # the ordered import takes it


@pytest.mark.parametrize("name", ["log4096", "mq6000_leaf32", "gauss5000_leaf16", "mixture6000_log"])
def test_gpu_built_operator(orc, name):
    xy, kern, leaf = _case(name)
    n = len(xy)
    x = np.random.default_rng(4).uniform(-1, 1, n)
    A = orc.dense_matrix(kern, xy)
    scale = np.abs(A) @ np.abs(x)
    yd = A @ x
    h = _lib()
    Hs = h.HODLR2D.build(dev(xy), kern, leaf, 1e-10, symmetric=True)
    e = np.abs(host(Hs.matvec(dev(x))) - yd)
    Is = Hs.info()
    Ho = h.HODLR2D.build(dev(xy), kern, leaf, 1e-10)
    Io = Ho.info()
    eo = np.abs(host(Ho.matvec(dev(x))) - yd)
    st_s = Is["u_elems"] + Is["v_elems"] + Is["d_elems"]
    st_o = Io["u_elems"] + Io["v_elems"] + Io["d_elems"]
    say(f"{name}: max row error / (|A||x|) symmetric {np.max(e / scale):.2e}, ordered {np.max(eo / scale):.2e}; "
        f"stored values {st_s / 1e6:.2f} M vs {st_o / 1e6:.2f} M")
    assert np.all(e <= 20 * 1e-10 * scale)
    assert Is["v_elems"] == 0
    # one pair of factors per pair, one dense block per leaf pair: about half
    # (the self blocks are stored whole)
    assert st_s <= 0.56 * st_o
    # the owners' ranks follow the oracle's (same pivoting rule, different rounding)
    O = orc.OracleH(xy, kern, leaf, 1e-10, symmetric=True)
    tab = O.il_table()
    assert Is["n_il"] == len(tab["tgt"])
    assert abs(Is["max_rank"] - int(np.max(np.where(tab["kind"] == 0, tab["rank"], 0)))) <= 3
    assert abs(Is["n_il_dense"] - int(np.sum(tab["kind"] == 1))) <= 0.01 * Is["n_il"] + 2


def test_zero_tolerance_equals_dense_product(orc):
    xy = np.random.default_rng(14).uniform(-1, 1, (1500, 2))
    x = np.random.default_rng(15).uniform(-1, 1, 1500)
    A = orc.dense_matrix(MQ, xy)
    H0 = _lib().HODLR2D.build(dev(xy), MQ, 16, 0.0, symmetric=True)
    assert H0.info()["n_il_dense"] == H0.info()["n_il"]
    e0 = np.abs(host(H0.matvec(dev(x))) - A @ x)
    assert np.all(e0 <= 1e-13 * (np.abs(A) @ np.abs(x)))


def test_export_round_trip(tmp_path):
    xy, kern, leaf = _case("mixture6000_log")
    h = _lib()
    H = h.HODLR2D.build(dev(xy), kern, leaf, 1e-10, symmetric=True)
    x = np.random.default_rng(5).uniform(-1, 1, len(xy))
    y = host(H.matvec(dev(x))).copy()
    p = tmp_path / "g.h2dx"
    H.export(p)
    # the ordered import applies the written mirrors as blocks of their own:
    # the same operator, other summation order
    Ho = h.HODLR2D.import_file(p)
    yo = host(Ho.matvec(dev(x)))
    assert np.linalg.norm(yo - y) <= 1e-13 * np.linalg.norm(y)
    # shared again: the same layout and order, the same bits
    Hs = h.HODLR2D.import_file(p, symmetric=True)
    assert np.array_equal(host(Hs.matvec(dev(x))), y)


def test_plain_solve_matches_oracle(orc, tmp_path):
    xy, kern, leaf = _case("mixture6000_log")
    O = orc.OracleH(xy, kern, leaf, 1e-10, symmetric=True)
    p = tmp_path / "o.h2dx"
    O.export(p)
    H = _lib().HODLR2D.import_file(p, symmetric=True)
    b = np.random.default_rng(7).uniform(-1, 1, len(xy))
    xo, it, rr, st = O.gmres(b, tol=1e-12)
    assert st == 0
    x, info = H.solve(dev(b), tol=1e-10)
    s = np.linalg.svd(orc.dense_matrix(kern, xy), compute_uv=False)
    cond = s[0] / s[-1]
    err = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
    say(f"symmetric GMRES: {info['iters']} its (oracle {it}), relres {info['relres']:.2e}, "
        f"error vs oracle {err:.2e}, cond {cond:.2f}")
    assert info["converged"] and abs(info["iters"] - it) <= 3
    assert err <= cond * (info["relres"] + rr)


def test_refusals():
    h = _lib()
    xy, kern, leaf = _case("mq6000_leaf32")
    for kw in ({"precs": ("fp16",)}, {"adaptive": True}):
        with pytest.raises(h.H2DError) as e:
            h.HODLR2D.build(dev(xy), kern, leaf, 1e-10, symmetric=True, **kw)
        assert e.value.code == h.H2D_EUNSUPPORTED
    with pytest.raises(h.H2DError) as e:
        h.HODLR2D.build(dev(xy), {"kind": "sep", "c": 3, "diag_mode": "formula"}, leaf, 1e-10, symmetric=True)
    assert e.value.code == h.H2D_EUNSUPPORTED
    # leaves above 64 points (300 points, leaf_max 100: four leaves of ~75)
    xy3 = np.random.default_rng(9).uniform(-1, 1, (300, 2))
    with pytest.raises(h.H2DError) as e:
        h.HODLR2D.build(dev(xy3), kern, 100, 1e-10, symmetric=True)
    assert e.value.code == h.H2D_EUNSUPPORTED
    H = h.HODLR2D.build(dev(xy), kern, leaf, 1e-10, symmetric=True)
    xd = dev(np.ones(len(xy)))
    for call in (H.bj_setup, lambda: H.solve(xd, precond="bj"), lambda: H.solve(xd, mode="refine"),
                 lambda: H.matvec_noalloc(xd), lambda: H.autotune(16), lambda: H.set_item_rows("b1_rows", 32)):
        with pytest.raises(h.H2DError) as e:
            call()
        assert e.value.code == h.H2D_EUNSUPPORTED


def test_full_size_rows_and_time(orc):
    """N = 2^20 multiquadric (the benchmark's workload), symmetric build:
    sampled rows against the oracle's exact O(N) rows within 10 tol of
    sum_j |A_ij x_j|, bitwise repeatable, and the product's time beside the
    ordered form's."""
    import torch
    h = _lib()
    xy, b, kern, leaf, tol = inputs.workload("mq1m")
    n = xy.shape[0]
    rows = np.sort(np.random.default_rng(78).choice(n, 32, replace=False))
    say("symmetric full-size build")
    H = h.HODLR2D.build(dev(xy), kern, leaf, tol, symmetric=True)
    I = H.info()
    x = dev(b)
    y1 = host(H.matvec(x)).copy()
    assert np.array_equal(host(H.matvec(x)), y1)
    say("oracle exact rows")
    ye = orc.dense_rows(kern, xy, b, rows)
    absrow = np.array([np.sum(np.abs(orc.entries(kern, xy, np.full(n, i), np.arange(n)) * b)) for i in rows])
    err = np.max(np.abs(y1[rows] - ye) / absrow)
    y = torch.empty_like(x)
    for _ in range(3):
        H.matvec(x, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        H.matvec(x, out=y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    stored = I["u_elems"] + I["d_elems"]
    say(f"symmetric N=2^20: {stored * 8 / 1e9:.2f} GB stored, {I['alg_bytes_fp64'] / 1e9:.2f} GB read per product, "
        f"{ms:.3f} ms, max row error {err:.2e}")
    assert err <= 10 * tol
