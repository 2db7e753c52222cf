"""Pins for the FP64 MLP reference: central finite differences of the loss
agree with the analytic gradient (the oracle the GPU training kernels are
checked against)."""
import numpy as np

from oracle import mlp


def test_finite_differences():
    rng = np.random.default_rng(0)
    w = rng.normal(0, 0.1, mlp.NPARAMS)
    B = 6
    X = rng.normal(size=(B, mlp.IN)); T = rng.normal(size=(B, mlp.OUT))
    M = (rng.uniform(size=(B, mlp.OUT)) < 0.7).astype(float)
    L, g = mlp.loss_grad(w, X, T, M)
    assert L == mlp.loss(w, X, T, M)
    idx = rng.choice(mlp.NPARAMS, 60, replace=False)
    # include every bias block and the last layer
    idx = np.concatenate([idx, [mlp.NPARAMS - 1, 256 * 192, 256 * 192 + 256 + 256 * 256 + 5]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(w); e[i] = h
        fd = (mlp.loss(w + e, X, T, M) - mlp.loss(w - e, X, T, M)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9


def test_pack_roundtrip():
    w = np.arange(mlp.NPARAMS, dtype=float)
    assert np.array_equal(mlp.pack(mlp.unpack(w)), w)
    assert mlp.NPARAMS == 131648
