"""Solves against the oracle's solution.

On the oracle's own factors (imported through h2d_import, FP16 and BF16
pools made from them), every solver form of the library -- plain FP64
GMRES, FP64 refinement around FP16 and BF16 inner solves, flexible GMRES
with block-Jacobi and with the learned preconditioner, and the chosen form
(FP16 refinement + learned preconditioner) -- is compared element by
element with the oracle's FP64 GMRES solution of the same operator taken to
relative residual 1e-12.

The bound: for two approximate solutions of A_hat x = b with relative
residuals r1, r2, |x1 - x2| <= cond(A_hat) (r1 + r2) |x| (2-norm), and the
max norm is at most the 2-norm.  cond is computed by numpy's SVD of the
dense kernel matrix at N = 4096 (1.62; the HODLR2D operator is within 1e-10
of it).  At N = 2^16 the dense SVD is out of reach; the log kernel with
diagonal N keeps its conditioning as N grows (1.66 at N = 1024, 1.62 at
4096), and the test takes 4 as its bound there.  Each result's error
against the oracle is printed: it is the per-result figure the precision
form states.
"""
import numpy as np
import pytest

from paper_2204_05536_amd import inputs
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

CASES = [("log4096", None), ("log1m", 1 << 16)]


def _lib():
    from paper_2204_05536_amd import hodlr2d
    return hodlr2d


@pytest.fixture(scope="module", params=CASES, ids=["log4096", "log65536"])
def case(request, orc, tmp_path_factory):
    name, n = request.param
    xy, b, kern, leaf, tol = inputs.workload(name, n=n)
    say(f"case {name} n={xy.shape[0]}: oracle build")
    O = orc.OracleH(xy, kern, leaf, tol)
    p = tmp_path_factory.mktemp("solve") / "o.h2dx"
    O.export(p)
    xo, it, rr, st = O.gmres(b, tol=1e-12)
    assert st == 0 and rr <= 1e-12, (it, rr, st)
    if xy.shape[0] <= 4096:
        s = np.linalg.svd(orc.dense_matrix(kern, xy), compute_uv=False)
        cond = s[0] / s[-1]
    else:
        cond = 4.0
    H = _lib().HODLR2D.import_file(p, precs=("fp16", "bf16"))
    say(f"case {name}: oracle GMRES {it} its relres {rr:.2e}, cond {cond:.3f}")
    return {"H": H, "b": b, "xo": xo, "rr": rr, "cond": cond, "name": name, "O": O}


def _check(case, x, info, tol, label):
    xo = case["xo"]
    x = host(x)
    e = x - xo
    err2 = np.linalg.norm(e) / np.linalg.norm(xo)
    errm = np.max(np.abs(e)) / np.max(np.abs(xo))
    bound = case["cond"] * (info["relres"] + case["rr"])
    say(f"{case['name']} {label}: its {info['iters']} outer {info['outer']} relres {info['relres']:.2e} | "
        f"vs oracle: 2-norm {err2:.2e}, max {errm:.2e} (bound {bound:.2e})")
    assert info["converged"] and info["relres"] <= tol, (label, info)
    # the residual the solver reports is the true FP64 residual of A_hat:
    # recompute it with the oracle's own product
    O = case["O"]
    b = case["b"]
    rt = np.linalg.norm(b - O.matvec(x)) / np.linalg.norm(b)
    assert rt <= 1.01 * tol and abs(rt - info["relres"]) <= 1e-3 * tol + 1e-14, (label, rt, info["relres"])
    assert err2 <= bound, (label, err2, bound)
    assert np.max(np.abs(e)) <= bound * np.linalg.norm(xo), (label, errm)
    return err2


def test_plain_fp64_matches_oracle(case):
    x, info = case["H"].solve(dev(case["b"]), tol=1e-10)
    _check(case, x, info, 1e-10, "plain FP64 GMRES to 1e-10")


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_refinement_to_1e10_matches_oracle(case, prec):
    """Half-precision factors, FP32 accumulation, FP64 refinement to 1e-10:
    the refined solution is within cond * 1e-10 of the oracle's."""
    x, info = case["H"].solve(dev(case["b"]), tol=1e-10, mode="refine", inner_prec=prec, inner_tol=1e-4)
    assert info["outer"] >= 2   # the half operator alone cannot reach 1e-10
    _check(case, x, info, 1e-10, f"refine {prec} to 1e-10")


def test_block_jacobi_fgmres_matches_oracle(case):
    H = case["H"]
    H.bj_setup()
    x, info = H.solve(dev(case["b"]), tol=1e-8, precond="bj")
    _check(case, x, info, 1e-8, "FGMRES + block-Jacobi to 1e-8")


def test_refine_fp16_block_jacobi_matches_oracle(case):
    H = case["H"]
    H.bj_setup()
    x, info = H.solve(dev(case["b"]), tol=1e-10, mode="refine", inner_prec="fp16", inner_tol=1e-4, precond="bj")
    _check(case, x, info, 1e-10, "refine fp16 + block-Jacobi to 1e-10")


def test_learned_preconditioner_forms_match_oracle(case):
    """The learned preconditioner trained on this operator, then FGMRES with
    it (1e-8) and the chosen form, FP16 refinement with it (1e-8 and
    1e-10): whatever the network does, the solutions must agree with the
    oracle's within the residual bound."""
    H = case["H"]
    H.bj_setup()
    info_t = H.mlp_train(n_solves=8, steps=300, batch=1024, lr=5e-4, seed=21)
    say("training", info_t)
    x, info = H.solve(dev(case["b"]), tol=1e-8, precond="mlp")
    _check(case, x, info, 1e-8, "FGMRES + MLP to 1e-8")
    for tol in (1e-8, 1e-10):
        x, info = H.solve(dev(case["b"]), tol=tol, mode="refine", inner_prec="fp16", inner_tol=1e-4, precond="mlp")
        _check(case, x, info, tol, f"chosen form (refine fp16 + MLP) to {tol:g}")
