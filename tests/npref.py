"""Independent numpy formulas used to pin the oracle (no oracle code here)."""
import numpy as np


def kernel_matrix(spec, X, Y=None, same=True):
    """K(X_i, Y_j) by numpy; when same, the diagonal follows spec's rule."""
    if Y is None:
        Y = X
    d = X[:, None, :] - Y[None, :, :]
    r = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)
    kind = spec["kind"]
    c = spec.get("c", 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        if kind == "log":
            K = np.log(r)
        elif kind == "invr":
            K = 1.0 / r
        elif kind == "mq":
            K = np.sqrt(1.0 + (r / c) ** 2)
        elif kind == "gauss":
            K = np.exp(-(r / c) ** 2)
        elif kind == "phi1":
            a = c
            small = (np.where(r > 0, r * np.log(np.where(r > 0, r, 1.0)), 0.0) - 1.0) / (a * np.log(a) - 1.0)
            K = np.where(r >= a, np.log(np.where(r > 0, r, 1.0)) / np.log(a), small)
        elif kind == "phi2":
            a = c
            K = np.where(r >= a, a / np.where(r > 0, r, 1.0), r / a)
        else:
            raise ValueError(kind)
    if same:
        n = X.shape[0]
        idx = np.arange(n)
        mode = spec.get("diag_mode", "formula")
        if mode == "replace":
            K[idx, idx] = spec["diag_value"]
        elif mode == "add":
            base = {"mq": 1.0, "gauss": 1.0}[kind]
            K[idx, idx] = base + spec["diag_value"]
    return K


def morton_np(ix, iy, level):
    """Bit-interleaved key: bit 2b = x bit b, bit 2b+1 = y bit b."""
    ix = np.asarray(ix, np.uint64); iy = np.asarray(iy, np.uint64)
    key = np.zeros_like(ix)
    for b in range(level):
        key |= ((ix >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        key |= ((iy >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    return key


def cells_np(v, R, level):
    """Cell index per coordinate by floor((v + R) 2^level / 2R), clamped to
    the top cell; exact for the dyadic test inputs used here."""
    c = np.floor((np.asarray(v) + R) * (2 ** level) / (2 * R)).astype(np.int64)
    return np.minimum(c, 2 ** level - 1)
