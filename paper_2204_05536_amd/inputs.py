"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path.

This module only draws numbers; it holds none of the HODLR2D arithmetic.
Every generator takes an explicit seed and uses numpy's PCG64
(``np.random.default_rng``), so the same call gives the same arrays on any
machine.  Shapes follow the paper's workloads: points in the square
[-1, 1]^2 (Section 5 uses [-1, 1]^2 throughout), Chebyshev grids (Section 5.1
and 5.2), and random right-hand sides.

Workloads (sizes and kernels as named by each function):
  * ``uniform_square``      i.i.d. uniform points in [-1, 1]^2
  * ``uniform_disc``        i.i.d. uniform points in the unit disc
  * ``gaussian_mixture``    4 equal clusters at (+-0.5, +-0.5), sigma 0.05,
                            draws outside [-1, 1]^2 rejected
  * ``chebyshev_grid``      sqrt(N) x sqrt(N) first-kind Chebyshev grid
  * ``rhs``                 entries uniform in [-1, 1]
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_square", "uniform_disc", "gaussian_mixture", "chebyshev_grid",
    "rhs", "batched_sizes", "workload", "batch_workload",
]


def uniform_square(n: int, rng: np.random.Generator) -> np.ndarray:
    """n x 2 float64 points, i.i.d. uniform in [-1, 1]^2 (row-major)."""
    return rng.uniform(-1.0, 1.0, size=(n, 2))


def uniform_disc(n: int, rng: np.random.Generator) -> np.ndarray:
    """n x 2 points uniform in the unit disc: radius sqrt(U), angle 2 pi U."""
    r = np.sqrt(rng.uniform(0.0, 1.0, size=n))
    th = rng.uniform(0.0, 2.0 * np.pi, size=n)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def gaussian_mixture(n: int, rng: np.random.Generator, sigma: float = 0.05) -> np.ndarray:
    """n x 2 points from 4 equal-weight Gaussians centred at (+-0.5, +-0.5).

    Draws falling outside [-1, 1]^2 are rejected and redrawn.
    """
    centres = np.array([[-0.5, -0.5], [0.5, -0.5], [0.5, 0.5], [-0.5, 0.5]])
    out = np.empty((0, 2))
    while out.shape[0] < n:
        m = n - out.shape[0]
        c = centres[rng.integers(0, 4, size=m)]
        p = c + sigma * rng.standard_normal(size=(m, 2))
        keep = np.all(np.abs(p) <= 1.0, axis=1)
        out = np.concatenate([out, p[keep]], axis=0)
    return np.ascontiguousarray(out[:n])


def chebyshev_grid(m: int) -> np.ndarray:
    """m*m points on the first-kind Chebyshev grid cos((2k-1) pi / 2m)^2."""
    k = np.arange(1, m + 1)
    c = np.cos((2 * k - 1) * np.pi / (2 * m))
    X, Y = np.meshgrid(c, c, indexing="xy")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel()], axis=1))


def rhs(n: int, rng: np.random.Generator, nrhs: int = 1) -> np.ndarray:
    """Right-hand side(s), entries uniform in [-1, 1].

    Returns shape (n,) for one RHS, else (nrhs, n): RHS r is row r, so that a
    C-contiguous array is column-major n x nrhs with leading dimension n.
    """
    if nrhs == 1:
        return rng.uniform(-1.0, 1.0, size=n)
    return rng.uniform(-1.0, 1.0, size=(nrhs, n))


def batched_sizes(count: int, rng: np.random.Generator,
                  lo: float = 1e4, hi: float = 5e5) -> np.ndarray:
    """Instance sizes N_i = round(exp(U(ln lo, ln hi)))."""
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)


# Named workloads.  Kernels are described by plain dicts so that this module
# holds no kernel arithmetic: kind, shape parameter c, diagonal rule.
def workload(name: str, n: int | None = None):
    """Return (points, rhs, kernel_spec, leaf, tol) for a named workload.

    ``n`` overrides the point count (same distribution and seed) so the
    same recipe can be run at reduced size.
      * "log4096":   log|x-y|, diagonal replaced by N, N=4096, seed 0
      * "mq1m":      multiquadric sqrt(1+(r/0.1)^2) + 1e-6 I, N=2^20, seed 1
      * "log1m":     log|x-y|, diagonal N, N=2^20, seed 2
    """
    if name == "log4096":
        seed, nn, spec = 0, 4096, ("log", 0.0, "replace", None)
    elif name == "mq1m":
        seed, nn, spec = 1, 1 << 20, ("mq", 0.1, "add", 1e-6)
    elif name == "log1m":
        seed, nn, spec = 2, 1 << 20, ("log", 0.0, "replace", None)
    else:
        raise ValueError(f"unknown workload {name!r}")
    if n is not None:
        nn = int(n)
    rng = np.random.default_rng(seed)
    xy = uniform_square(nn, rng)
    b = rhs(nn, rng)
    kind, c, dmode, dval = spec
    if dval is None:
        dval = float(nn)
    kern = {"kind": kind, "c": c, "diag_mode": dmode, "diag_value": dval}
    return xy, b, kern, 64, 1e-10


def batch_workload(count: int = 64, seed: int = 3, lo: float = 1e4, hi: float = 5e5, nrhs: int = 16):
    """Independent instances for the batched product.

    Returns (instances, kernel_spec, leaf, tol); instance i is a pair
    (points N_i x 2, right-hand sides nrhs x N_i).  N_i is log-uniform in
    [lo, hi]; even instances are uniform in the unit disc, odd ones the
    4-cluster Gaussian mixture (sigma 0.05).  Kernel: Gaussian RBF with
    shape 0.05 plus 1e-4 on the diagonal.
    """
    rng = np.random.default_rng(seed)
    sizes = batched_sizes(count, rng, lo, hi)
    inst = []
    for i in range(count):
        n = int(sizes[i])
        xy = uniform_disc(n, rng) if i % 2 == 0 else gaussian_mixture(n, rng)
        inst.append((xy, rhs(n, rng, nrhs) if nrhs > 1 else rhs(n, rng)))
    kern = {"kind": "gauss", "c": 0.05, "diag_mode": "add", "diag_value": 1e-4}
    return inst, kern, 64, 1e-10
