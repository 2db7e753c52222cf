"""Batched products replayed from one captured HIP graph, and the phase-A
item-size tuner: every replay must equal the eager product of each
instance, and a tuned handle must still agree with the oracle's factors."""
import numpy as np
import pytest
import torch

from paper_2204_05536_amd import inputs
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2204_05536_amd import hodlr2d
    return hodlr2d


def _instances(count, nrhs, seed=5):
    inst, kern, leaf, tol = inputs.batch_workload(count, seed, 1500, 30000, nrhs)
    hs = [_lib().HODLR2D.build(dev(xy), kern, leaf, tol) for xy, _ in inst]
    return inst, hs


@pytest.mark.parametrize("nrhs", [1, 16, 20])
def test_graph_replays_match_eager(nrhs):
    inst, hs = _instances(7, nrhs)
    xs = [dev(X) for _, X in inst]
    ys = [torch.zeros_like(x) for x in xs]
    B = _lib().Batch(hs, xs, ys)
    rng = np.random.default_rng(11)
    for rep in range(3):
        say(f"batch nrhs={nrhs} replay {rep}")
        if rep:   # new values in the bound buffers, written by ordinary eager work
            for x in xs:
                x.copy_(torch.from_numpy(rng.uniform(-1, 1, tuple(x.shape))).to(x.device))
        B.launch()
        torch.cuda.synchronize()
        for i, H in enumerate(hs):
            ye = host(H.matvec(xs[i]))
            assert np.array_equal(host(ys[i]), ye), (rep, i)
        for y in ys:
            y.zero_()
    B.close()


def test_same_handle_twice_in_batch():
    inst, hs = _instances(2, 16)
    x0 = dev(inst[0][1])
    x1 = dev(np.random.default_rng(2).uniform(-1, 1, inst[0][1].shape))
    y0, y1, y2 = (torch.zeros_like(x0) for _ in range(3))
    xb = dev(inst[1][1])
    yb = torch.zeros_like(xb)
    B = _lib().Batch([hs[0], hs[1], hs[0]], [x0, xb, x1], [y0, yb, y1])
    for rep in range(2):
        B.launch()
        torch.cuda.synchronize()
        assert np.array_equal(host(y0), host(hs[0].matvec(x0)))
        assert np.array_equal(host(y1), host(hs[0].matvec(x1)))
        assert np.array_equal(host(yb), host(hs[1].matvec(xb)))
    B.close()


def test_autotune_keeps_results(orc, tmp_path):
    xy, b, kern, leaf, tol = inputs.workload("log4096")
    O = orc.OracleH(xy, kern, leaf, tol)
    p = tmp_path / "o.h2dx"
    O.export(p)
    H = _lib().HODLR2D.import_file(p)
    X = np.random.default_rng(6).uniform(-1, 1, (16, xy.shape[0]))
    chosen, ms = H.autotune(16)
    say(f"autotune chose {chosen}, ms {ms}")
    assert chosen["mr_rows"] in (128, 256, 512)
    assert all(v > 0 for v in ms.values())
    chosen1, ms1 = H.autotune(1)
    say(f"autotune (1 RHS) chose {chosen1}, ms {ms1}")
    assert chosen1["a_rows"] in (128, 256, 512) and chosen1["b1_rows"] in (16, 32, 64)
    assert chosen1["b2_rows"] in (16, 32, 64)
    Y = host(H.matvec(dev(X)))
    y1 = host(H.matvec(dev(X[3])))
    for r in range(16):
        yo = O.matvec(X[r])
        assert np.linalg.norm(Y[r] - yo) <= 1e-12 * np.linalg.norm(yo)
    assert np.linalg.norm(y1 - O.matvec(X[3])) <= 1e-12 * np.linalg.norm(y1)


@pytest.mark.parametrize("rows,b1", [(16, 16), (128, 32), (256, 64)])
def test_item_size_changes_schedule_not_result(rows, b1):
    """Smaller phase-A items split more V blocks into partial sums, smaller
    phase-B1 slices add column groups; the product (single- and multi-RHS)
    must agree with the default schedule to rounding."""
    rng = np.random.default_rng(rows)
    xy = inputs.uniform_square(30000, rng)
    spec = {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}
    H = _lib().HODLR2D.build(dev(xy), spec, 64, 1e-10)
    x = rng.uniform(-1, 1, (16, 30000))
    y_ref = host(H.matvec(dev(x)))
    y1_ref = host(H.matvec(dev(x[0])))
    H.set_item_rows("a_rows", rows)
    H.set_item_rows("mr_rows", max(rows // 2, 16))
    H.set_item_rows("b1_rows", b1)
    y = host(H.matvec(dev(x)))
    y1 = host(H.matvec(dev(x[0])))
    assert np.linalg.norm(y - y_ref) <= 1e-14 * np.linalg.norm(y_ref)
    assert np.linalg.norm(y1 - y1_ref) <= 1e-14 * np.linalg.norm(y1_ref)


@pytest.mark.parametrize("b2", [16, 32])
def test_leaf_chunk_rows_change_schedule_not_result(b2):
    """Leaves of up to 200 points split into chunks of 16 or 32 rows (several
    column groups per wave) instead of 64: the FP64 product agrees with the
    default schedule to rounding, the FP16 one to FP32 rounding."""
    rng = np.random.default_rng(40 + b2)
    xy = inputs.uniform_square(20000, rng)
    spec = {"kind": "mq", "c": 0.1, "diag_mode": "add", "diag_value": 1e-6}
    H = _lib().HODLR2D.build(dev(xy), spec, 200, 1e-10, precs=("fp16",))
    x = dev(rng.uniform(-1, 1, 20000))
    y_ref, yh_ref = host(H.matvec(x)), host(H.matvec(x, prec="fp16"))
    H.set_item_rows("b2_rows", b2)
    y, yh = host(H.matvec(x)), host(H.matvec(x, prec="fp16"))
    assert np.linalg.norm(y - y_ref) <= 1e-14 * np.linalg.norm(y_ref)
    assert np.linalg.norm(yh - yh_ref) <= 1e-6 * np.linalg.norm(yh_ref)
    # the no-allocation product runs the same schedule
    assert np.array_equal(host(H.matvec_noalloc(x)), y)
