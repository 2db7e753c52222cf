"""The oracle's export round-trips: the dense operator rebuilt from the file
applies exactly the oracle's Algorithm 2 (to summation-order rounding)."""
import numpy as np

from tests import h2dfile


def test_oracle_export_roundtrip(orc, tmp_path):
    rng = np.random.default_rng(31)
    xy = rng.uniform(-1, 1, (700, 2)); x = rng.uniform(-1, 1, 700)
    spec = {"kind": "log", "diag_mode": "replace", "diag_value": 700.0}
    H = orc.OracleH(xy, spec, 16, 1e-8)
    p = tmp_path / "h.h2dx"
    H.export(p)
    F = h2dfile.read(p)
    assert F["kappa"] == H.kappa and np.array_equal(F["perm"], H.perm())
    tab = H.il_table()
    assert np.array_equal(F["il_rank"], tab["rank"]) and np.array_equal(F["il_kind"], tab["kind"])
    A = h2dfile.dense_operator(F)
    y = H.matvec(x)
    assert np.linalg.norm(A @ x - y) <= 1e-13 * np.linalg.norm(y)
