"""FP64 reference of the per-leaf MLP preconditioner's forward and backward
passes (plain numpy matrix products) — TEST INFRASTRUCTURE ONLY.

Network 192 -> 256 (ReLU) -> 256 (ReLU) -> 64, weights packed
[W1 (256 x 192), b1, W2 (256 x 256), b2, W3 (64 x 256), b3] row-major;
loss = sum M (out - T)^2 / (2 sum M).  Pinned by central finite differences
(tests/test_oracle_mlp.py)."""
import numpy as np

IN, HID, OUT = 192, 256, 64
SIZES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (OUT, HID)), ("b3", (OUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(w):
    out, o = {}, 0
    for name, shp in SIZES:
        k = int(np.prod(shp))
        out[name] = np.asarray(w[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(p):
    return np.concatenate([p[name].ravel() for name, _ in SIZES])


def forward(w, X):
    p = unpack(w)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    out = h2 @ p["W3"].T + p["b3"]
    return out, (X, z1, h1, z2, h2)


def loss(w, X, T, M):
    out, _ = forward(w, X)
    return float(np.sum(M * (out - T) ** 2) / (2.0 * max(1.0, np.sum(M))))


def loss_grad(w, X, T, M):
    p = unpack(w)
    out, (X, z1, h1, z2, h2) = forward(w, X)
    cnt = max(1.0, np.sum(M))
    d = M * (out - T) / cnt
    g = {"W3": d.T @ h2, "b3": d.sum(0)}
    d2 = (d @ p["W3"]) * (z2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * (z1 > 0)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(0)
    return float(np.sum(M * (out - T) ** 2) / (2.0 * cnt)), pack(g)
