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


def test_single_path_by_hand():
    """One nonzero weight per layer: the forward pass reduces to scalar
    arithmetic written out here, including both ReLU branches."""
    p = {name: np.zeros(shp) for name, shp in mlp.SIZES}
    p["W1"][3, 130] = 2.0; p["b1"][3] = -0.5
    p["W2"][7, 3] = -1.5; p["b2"][7] = 4.0
    p["W3"][11, 7] = 0.25; p["b3"][11] = 1.0; p["b3"][0] = -2.0
    w = mlp.pack(p)
    for xv in (1.0, 0.1, -3.0):
        X = np.zeros((1, mlp.IN)); X[0, 130] = xv
        h1 = max(2.0 * xv - 0.5, 0.0)
        h2 = max(-1.5 * h1 + 4.0, 0.0)
        out, _ = mlp.forward(w, X)
        expect = np.zeros(mlp.OUT); expect[11] = 1.0 + 0.25 * h2; expect[0] = -2.0
        assert np.array_equal(out[0], expect), xv


def test_zero_last_layer_loss_and_mask():
    """With W3 = b3 = 0 the output is 0, so the loss is the masked mean of
    T^2 / 2; masked-out slots contribute nothing whatever their target."""
    rng = np.random.default_rng(1)
    w = rng.normal(0, 0.1, mlp.NPARAMS)
    p = mlp.unpack(w); p["W3"][:] = 0.0; p["b3"][:] = 0.0
    w = mlp.pack(p)
    X = rng.normal(size=(5, mlp.IN)); T = rng.normal(size=(5, mlp.OUT))
    M = (rng.uniform(size=(5, mlp.OUT)) < 0.5).astype(float)
    L = mlp.loss(w, X, T, M)
    assert abs(L - np.sum(M * T * T) / (2 * M.sum())) <= 1e-15 * L
    T2 = T + 1e3 * (1 - M)
    assert mlp.loss(w, X, T2, M) == L
    # only the last layer's gradient can be nonzero at the first step
    _, g = mlp.loss_grad(w, X, T, M)
    n3 = mlp.OUT * mlp.HID + mlp.OUT
    assert np.count_nonzero(g[:-n3]) == 0
    assert np.count_nonzero(g[-n3:]) > 0
