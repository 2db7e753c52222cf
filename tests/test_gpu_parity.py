"""GPU parity: the HIP library against the CPU oracle.

  * tree, permutation, level tables and block lists: bit-exact;
  * matvec on the oracle's own factors (imported): 1e-12 relative in FP64;
  * GPU-built factors: the operator within the ACA tolerance of the dense
    product, ranks close to the oracle's;
  * bitwise repeatability (no atomics on the hot path).
"""
import numpy as np
import pytest

from paper_2204_05536_amd import inputs
from tests import h2dfile, npref
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

MQ = {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}
GA = {"kind": "gauss", "c": 0.05, "diag_mode": "add", "diag_value": 1e-4}


def _lib():
    from paper_2204_05536_amd import hodlr2d
    return hodlr2d


def _cases():
    rng = np.random.default_rng(100)
    c = []
    xy, b, k, leaf, tol = inputs.workload("log4096")
    c.append(("log4096", xy, k, leaf, tol))
    c.append(("mix3000_leaf16", inputs.gaussian_mixture(3000, rng), MQ, 16, 1e-10))
    c.append(("disc5000_leaf32", inputs.uniform_disc(5000, rng), GA, 32, 1e-10))
    c.append(("one_point", np.array([[0.3, -0.2]]), MQ, 64, 1e-10))
    c.append(("single_leaf_64", rng.uniform(-1, 1, (64, 2)), MQ, 64, 1e-10))
    c.append(("ragged_1337_leaf7", rng.uniform(-1, 1, (1337, 2)), MQ, 7, 1e-10))
    # leaves above 64 points: several 64-row chunks per leaf box
    c.append(("unif4000_leaf200", rng.uniform(-1, 1, (4000, 2)), MQ, 200, 1e-10))
    # points in the top half of B only: the two level-1 boxes share an edge,
    # so with kappa = 2 no block sits above the leaf level's parents and
    # every phase-B1 walk (and half-pool table) of a level-1 box is empty
    c.append(("top_half_300", np.stack([rng.uniform(-1, 1, 300), rng.uniform(0.01, 1, 300)], 1), MQ, 64, 1e-10))
    # points on cell boundaries, on the top / right edge of B, and at 0
    g = np.array([[-1.0, -1.0], [1.0, 1.0], [0.0, 0.0], [0.5, -0.5], [-0.5, 0.5], [1.0, -1.0], [-1.0, 1.0],
                  [0.25, 0.75], [0.0, 1.0], [1.0, 0.0]])
    c.append(("boundaries", np.concatenate([g, rng.uniform(-1, 1, (300, 2))]), MQ, 4, 1e-10))
    c.append(("cheb_40x40_leaf25", inputs.chebyshev_grid(40), {"kind": "invr", "diag_mode": "replace",
                                                                  "diag_value": 0.0}, 25, 1e-12))
    # the paper's RBF kernels (Section 5.2): a = 0.001, beta = N on the diagonal
    for kind in ("phi1", "phi2"):
        c.append((f"cheb_30x30_{kind}_leaf25", inputs.chebyshev_grid(30),
                  {"kind": kind, "c": 1e-3, "diag_mode": "replace", "diag_value": 900.0}, 25, 1e-12))
    # a Gaussian so narrow that K underflows to exactly 0 beyond r = 0.14:
    # blocks with zero rows before the first cross and after the last one
    c.append(("gauss_c0.005_unif4000_leaf16", rng.uniform(-1, 1, (4000, 2)),
              {"kind": "gauss", "c": 0.005, "diag_mode": "add", "diag_value": 0.3}, 16, 1e-10))
    return c


CASES = _cases()


def _compare_structure(F, O):
    assert F["kappa"] == O.kappa
    assert F["R"] == O.R
    assert np.array_equal(F["perm"], O.perm())
    for l in range(O.kappa + 1):
        L = O.level(l)
        for f in ("key", "begin", "count", "parent"):
            assert np.array_equal(F["levels"][l][f].astype(np.int64), L[f].astype(np.int64)), (l, f)
    t, s = O.near_table()
    assert np.array_equal(F["near_tgt"], t) and np.array_equal(F["near_src"], s)
    tab = O.il_table()
    for f, g in (("il_level", "level"), ("il_tgt", "tgt"), ("il_src", "src")):
        assert np.array_equal(F[f].astype(np.int64), tab[g].astype(np.int64)), f


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_structure_bit_exact(orc, tmp_path, case):
    name, xy, k, leaf, tol = case
    say("structure", name, xy.shape)
    H = _lib().HODLR2D.build(dev(xy), k, leaf, tol)
    p = tmp_path / "g.h2dx"
    H.export(p, factors=False)
    F = h2dfile.read(p)
    O = orc.OracleH(xy, k, leaf, tol, factors=False)
    _compare_structure(F, O)


U16 = 2.0 ** -11   # unit roundoff of FP16
UBF = 2.0 ** -8    # unit roundoff of BF16


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_matvec_on_oracle_factors(orc, tmp_path, case):
    """Identical H on both sides: only the summation order differs in FP64.
    The FP16 / BF16 pools made from the same factors (values rounded to the
    half format, FP32 accumulation): every row within 4 u of
    sum_j |A_ij x_j|.  Odd box sizes, odd ranks and leaves above 64 points
    in these cases exercise the half kernels' paired loads, whose value past
    a block's end is read and dropped."""
    name, xy, k, leaf, tol = case
    say("import-matvec", name)
    O = orc.OracleH(xy, k, leaf, tol)
    p = tmp_path / "o.h2dx"
    O.export(p)
    H = _lib().HODLR2D.import_file(p, precs=("fp16", "bf16"))
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, xy.shape[0])
    yo = O.matvec(x)
    yg = host(H.matvec(dev(x)))
    assert np.linalg.norm(yg - yo) <= 1e-12 * np.linalg.norm(yo)
    assert np.max(np.abs(yg - yo)) <= 1e-12 * np.max(np.abs(yo))
    absrow = np.abs(npref.kernel_matrix(k, xy)) @ np.abs(x)
    for prec, u in (("fp16", U16), ("bf16", UBF)):
        yh = host(H.matvec(dev(x), prec=prec))
        err = np.abs(yh - yo) / absrow
        say(prec, "max row error / sum|A x|", err.max())
        assert np.all(np.isfinite(yh)) and err.max() <= 4 * u, prec


@pytest.mark.parametrize("case", CASES[:3] + CASES[5:], ids=[c[0] for c in CASES[:3] + CASES[5:]])
def test_gpu_built_operator_accuracy(orc, tmp_path, case):
    """GPU-built factors: |A_hat x - A x| within 20 tol of |A_off x|, the
    oracle's own operator within the same bound, kinds equal and ranks
    within +-3 of the oracle's."""
    name, xy, k, leaf, tol = case
    say("gpu-built", name)
    H = _lib().HODLR2D.build(dev(xy), k, leaf, tol)
    O = orc.OracleH(xy, k, leaf, tol)
    x = np.random.default_rng(8).uniform(-1, 1, xy.shape[0])
    A = npref.kernel_matrix(k, xy)
    Aoff = A - np.diag(np.diag(A))
    ref = np.linalg.norm(Aoff @ x)
    yg = host(H.matvec(dev(x)))
    yo = O.matvec(x)
    bound = max(20 * tol, 1e-13) * ref
    assert np.linalg.norm(yo - A @ x) <= bound
    assert np.linalg.norm(yg - A @ x) <= bound
    p = tmp_path / "g.h2dx"
    H.export(p, factors=False)
    F = h2dfile.read(p)
    tab = O.il_table()
    same_kind = F["il_kind"] == tab["kind"]
    assert same_kind.mean() >= 0.99
    lr = same_kind & (tab["kind"] == 0)
    assert np.all(np.abs(F["il_rank"][lr] - tab["rank"][lr]) <= 3)


def test_repeatable_bits():
    xy, b, k, leaf, tol = inputs.workload("log4096")
    H = _lib().HODLR2D.build(dev(xy), k, leaf, tol)
    x = dev(b)
    y1 = host(H.matvec(x)).copy()
    y2 = host(H.matvec(x))
    assert np.array_equal(y1, y2)
    H2 = _lib().HODLR2D.build(dev(xy), k, leaf, tol)
    assert np.array_equal(y1, host(H2.matvec(x)))


def test_zero_tolerance_is_dense():
    rng = np.random.default_rng(9)
    xy = rng.uniform(-1, 1, (1500, 2)); x = rng.uniform(-1, 1, 1500)
    spec = {"kind": "log", "diag_mode": "replace", "diag_value": 1500.0}
    H = _lib().HODLR2D.build(dev(xy), spec, 16, 0.0)
    assert H.info()["n_il_dense"] == H.info()["n_il"]
    A = npref.kernel_matrix(spec, xy)
    assert np.linalg.norm(host(H.matvec(dev(x))) - A @ x) <= 1e-13 * np.linalg.norm(A @ x)


def test_error_statuses():
    h = _lib()
    xy = np.array([[0.1, 0.2], [0.5, 0.5], [0.1, 0.2]])
    with pytest.raises(h.H2DError) as e:
        h.HODLR2D.build(dev(xy), {"kind": "log", "diag_mode": "replace", "diag_value": 3.0}, 8, 1e-10)
    assert e.value.code == h.H2D_EDUP
    with pytest.raises(h.H2DError) as e:
        h.HODLR2D.build(dev(np.array([[0.0, np.nan]])), MQ, 8, 1e-10)
    assert e.value.code == h.H2D_EINVAL
    with pytest.raises(h.H2DError) as e:
        h.HODLR2D.build(dev(xy), {"kind": "mq", "c": -1.0, "diag_mode": "add", "diag_value": 0.0}, 8, 1e-10)
    assert e.value.code == h.H2D_EINVAL
    H = h.HODLR2D.build(dev(xy), MQ, 8, 1e-10)
    with pytest.raises(h.H2DError) as e:
        H.matvec(dev(np.ones(3)), prec="fp16")
    assert e.value.code == h.H2D_EUNSUPPORTED
    # empty input, no right-hand sides, a leading dimension below n
    import ctypes as C
    import torch
    L = h.load()
    k = h.kernel_spec(MQ)
    out = C.c_void_p()
    strm = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.h2d_build(C.c_void_p(dev(xy).data_ptr()), 0, C.byref(k), 8, 1e-10, 0, strm, C.byref(out)) == h.H2D_EINVAL
    assert L.h2d_build(None, 3, C.byref(k), 8, 1e-10, 0, strm, C.byref(out)) == h.H2D_EINVAL
    xd = dev(np.ones(3)); yd = dev(np.zeros(3))
    ptr = lambda t: C.c_void_p(t.data_ptr())
    assert L.h2d_matvec(H._h, ptr(xd), ptr(yd), 0, 3, 0, strm) == h.H2D_EINVAL
    assert L.h2d_matvec(H._h, ptr(xd), ptr(yd), 1, 2, 0, strm) == h.H2D_EINVAL
    assert L.h2d_matvec(H._h, None, ptr(yd), 1, 3, 0, strm) == h.H2D_EINVAL
    # 65 coincident points cannot be split by any depth
    with pytest.raises(h.H2DError) as e:
        h.HODLR2D.build(dev(np.zeros((65, 2))), MQ, 64, 1e-10)
    assert e.value.code == h.H2D_EDEPTH


def test_solve_plain_log4096(orc):
    xy, b, k, leaf, tol = inputs.workload("log4096")
    H = _lib().HODLR2D.build(dev(xy), k, leaf, tol)
    x, info = H.solve(dev(b), tol=1e-8, restart=50)
    assert info["converged"] and info["relres"] <= 1e-8
    O = orc.OracleH(xy, k, leaf, tol)
    xo, it, rr, st = O.gmres(b, 1e-8, 50, 500)
    assert abs(info["iters"] - it) <= 1
    A = npref.kernel_matrix(k, xy)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(host(x) - xd) <= 1e-7 * np.linalg.norm(xd)


def test_forced_allocation_failures_report_enomem():
    """H2D_TEST_FAIL_ALLOC=k makes the k-th device allocation fail: every
    such failure during a build surfaces as H2D_ENOMEM with the handle left
    unset, nothing stays allocated, and a later build works."""
    import os
    import torch
    h = _lib()
    xy, b, kern, leaf, tol = inputs.workload("log4096", n=1500)
    xd, bd = dev(xy), dev(b)
    ref = host(h.HODLR2D.build(xd, kern, leaf, tol, precs=("fp16",)).matvec(bd))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    try:
        for k in (1, 3, 7, 15, 30):
            os.environ["H2D_TEST_FAIL_ALLOC"] = str(k)
            with pytest.raises(h.H2DError) as e:
                h.HODLR2D.build(xd, kern, leaf, tol, precs=("fp16",))
            assert e.value.code == h.H2D_ENOMEM, (k, e.value)
            del os.environ["H2D_TEST_FAIL_ALLOC"]
    finally:
        os.environ.pop("H2D_TEST_FAIL_ALLOC", None)
    torch.cuda.synchronize()
    assert abs(torch.cuda.mem_get_info()[0] - free0) <= 64 << 20
    y = host(h.HODLR2D.build(xd, kern, leaf, tol, precs=("fp16",)).matvec(bd))
    assert np.array_equal(y, ref)
