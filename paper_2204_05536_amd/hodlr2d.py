"""Python binding of the HODLR2D C ABI (include/h2d.h).

Argument marshalling only: every step of build, matvec and solve runs in the
HIP library ``libh2d.so``.  Device memory and streams come from PyTorch
(ROCm); tensors are passed to the library as raw device pointers together
with the current stream.  The library must have been built (``build()`` in
``__graft_entry__`` or ``python -m paper_2204_05536_amd.build``); there is
no fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # loads the ROCm HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libh2d.so")

# enums mirrored from include/h2d.h
H2D_OK, H2D_EINVAL, H2D_ENOMEM, H2D_EDEVICE, H2D_EDUP, H2D_ENOCONV, H2D_EUNSUPPORTED, H2D_EDEPTH = range(8)
KINDS = {"log": 0, "invr": 1, "mq": 2, "gauss": 3, "phi1": 4, "phi2": 5, "sep": 6}
DIAG = {"replace": 0, "add": 1, "formula": 2}
PREC = {"fp64": 0, "fp16": 1, "bf16": 2}
SOLVE_PLAIN, SOLVE_REFINE = 0, 1
BUILD_ADAPTIVE = 1 << 8
BUILD_SYMMETRIC = 1 << 9
PRECOND = {"none": 0, "bj": 1, "mlp": 2}

EXPORTED = ["h2d_build", "h2d_matvec", "h2d_matvec_noalloc", "h2d_solve", "h2d_info", "h2d_export", "h2d_import",
            "h2d_profile_enable", "h2d_profile_read", "h2d_bj_setup", "h2d_precond_apply",
            "h2d_mlp_train", "h2d_mlp_weights", "h2d_mlp_loss_grad", "h2d_autotune", "h2d_set_item_rows", "h2d_batch_create",
            "h2d_batch_launch", "h2d_batch_destroy", "h2d_destroy", "h2d_last_error"]
MLP_PARAMS = 131648
MLP_PARAMS_PATCH = 328256
PHASES = ["gather", "phaseA", "reduce", "phaseB", "combine"]


class H2DError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"h2d status {code}: {msg}")
        self.code = code


class h2d_kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("diag_mode", C.c_int32), ("c", C.c_double), ("diag_value", C.c_double)]


class h2d_solve_opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("restart", C.c_int32), ("max_iter", C.c_int32), ("inner_prec", C.c_int32),
                ("inner_tol", C.c_double), ("max_outer", C.c_int32), ("precond", C.c_int32)]


class h2d_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer", C.c_int32), ("relres", C.c_double), ("seconds", C.c_double),
                ("fallback_at", C.c_int32), ("pad", C.c_int32)]


class h2d_stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("kappa", C.c_int32), ("leaf_max", C.c_int32), ("R", C.c_double),
                ("tol", C.c_double), ("n_near", C.c_int64), ("n_il", C.c_int64), ("n_il_dense", C.c_int64),
                ("max_rank", C.c_int64), ("sum_rank", C.c_int64), ("u_elems", C.c_int64), ("v_elems", C.c_int64),
                ("d_elems", C.c_int64), ("alg_bytes_fp64", C.c_double), ("alg_bytes_half", C.c_double),
                ("flops", C.c_double), ("build_seconds", C.c_double), ("prec_mask", C.c_uint32),
                ("pad", C.c_int32)]


class h2d_profile(C.Structure):
    _fields_ = [("count", C.c_int32), ("prec", C.c_int32), ("ms", C.c_double * 5), ("bytes", C.c_double * 5)]


class h2d_mlp_train_opts(C.Structure):
    _fields_ = [("n_solves", C.c_int32), ("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("seed", C.c_uint64), ("solve_tol", C.c_double), ("target", C.c_int32), ("input", C.c_int32)]


class h2d_mlp_train_info(C.Structure):
    _fields_ = [("seconds_data", C.c_double), ("seconds_train", C.c_double), ("loss_first", C.c_float),
                ("loss_last", C.c_float), ("n_samples", C.c_int32), ("solves_converged", C.c_int32),
                ("scale", C.c_double)]


_lib = None


def load():
    """Load libh2d.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} missing (run paper_2204_05536_amd/build.py)")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.h2d_build.argtypes = [P, C.c_int64, C.POINTER(h2d_kernel), C.c_int32, C.c_double, C.c_uint32, P,
                            C.POINTER(P)]
    L.h2d_build.restype = C.c_int
    L.h2d_matvec.argtypes = [P, P, P, C.c_int32, C.c_int64, C.c_int32, P]
    L.h2d_matvec.restype = C.c_int
    L.h2d_matvec_noalloc.argtypes = [P, P, P, C.c_int32, P]
    L.h2d_matvec_noalloc.restype = C.c_int
    L.h2d_solve.argtypes = [P, P, P, C.c_double, C.POINTER(h2d_solve_opts), C.POINTER(h2d_solve_info), P]
    L.h2d_solve.restype = C.c_int
    L.h2d_info.argtypes = [P, C.POINTER(h2d_stats)]
    L.h2d_info.restype = C.c_int
    L.h2d_export.argtypes = [P, C.c_char_p, C.c_uint32]
    L.h2d_export.restype = C.c_int
    L.h2d_import.argtypes = [C.c_char_p, C.c_uint32, P, C.POINTER(P)]
    L.h2d_import.restype = C.c_int
    L.h2d_profile_enable.argtypes = [P, C.c_int32]
    L.h2d_profile_enable.restype = C.c_int
    L.h2d_profile_read.argtypes = [P, C.POINTER(h2d_profile)]
    L.h2d_profile_read.restype = C.c_int
    L.h2d_bj_setup.argtypes = [P, P]
    L.h2d_bj_setup.restype = C.c_int
    L.h2d_precond_apply.argtypes = [P, C.c_int32, P, P, P]
    L.h2d_precond_apply.restype = C.c_int
    L.h2d_mlp_train.argtypes = [P, C.POINTER(h2d_mlp_train_opts), C.POINTER(h2d_mlp_train_info), P]
    L.h2d_mlp_train.restype = C.c_int
    L.h2d_mlp_weights.argtypes = [P, P, P, C.POINTER(C.c_double), P]
    L.h2d_mlp_weights.restype = C.c_int
    L.h2d_mlp_loss_grad.argtypes = [P, P, P, P, C.c_int32, C.POINTER(C.c_float), P, P]
    L.h2d_mlp_loss_grad.restype = C.c_int
    L.h2d_autotune.argtypes = [P, C.c_int32, P, C.POINTER(C.c_int32), C.POINTER(C.c_float)]
    L.h2d_autotune.restype = C.c_int
    L.h2d_set_item_rows.argtypes = [P, C.c_int32, C.c_int32, P]
    L.h2d_set_item_rows.restype = C.c_int
    L.h2d_batch_create.argtypes = [C.POINTER(P), C.c_int32, C.c_int32, C.POINTER(P), C.POINTER(P),
                                   C.POINTER(C.c_int64), C.POINTER(P)]
    L.h2d_batch_create.restype = C.c_int
    L.h2d_batch_launch.argtypes = [P, P]
    L.h2d_batch_launch.restype = C.c_int
    L.h2d_batch_destroy.argtypes = [P]
    L.h2d_batch_destroy.restype = None
    L.h2d_destroy.argtypes = [P]
    L.h2d_destroy.restype = None
    L.h2d_last_error.argtypes = []
    L.h2d_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(st):
    if st != H2D_OK:
        raise H2DError(st, load().h2d_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA/HIP tensor")
    return C.c_void_p(t.data_ptr())


def kernel_spec(spec: dict) -> h2d_kernel:
    return h2d_kernel(KINDS[spec["kind"]], DIAG[spec.get("diag_mode", "formula")], float(spec.get("c", 0.0)),
                      float(spec.get("diag_value", 0.0)))


def prec_mask(*precs):
    m = 1
    for p in precs:
        m |= 1 << PREC[p]
    return m


class HODLR2D:
    """A built HODLR2D operator on the current GPU.

    ``HODLR2D.build(xy, kernel, leaf_max, tol, precs)``: xy is an (N, 2)
    float64 tensor on the GPU; kernel a dict (kind, c, diag_mode,
    diag_value).  ``matvec(x)`` returns A_hat x, ``solve(b, tol)`` returns x.
    """

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def build(cls, xy, kernel, leaf_max=64, tol=1e-10, precs=(), adaptive=False, symmetric=False):
        L = load()
        xy = xy.contiguous()
        h = C.c_void_p()
        k = kernel_spec(kernel)
        flags = prec_mask(*precs) | (BUILD_ADAPTIVE if adaptive else 0) | (BUILD_SYMMETRIC if symmetric else 0)
        _check(L.h2d_build(_dev_f64(xy, "xy"), xy.shape[0], C.byref(k), int(leaf_max), float(tol),
                           flags, _stream(), C.byref(h)))
        return cls(h)

    @classmethod
    def import_file(cls, path, precs=(), symmetric=False):
        L = load()
        h = C.c_void_p()
        flags = prec_mask(*precs) | (BUILD_SYMMETRIC if symmetric else 0)
        _check(L.h2d_import(str(path).encode(), flags, _stream(), C.byref(h)))
        return cls(h)

    def close(self):
        if getattr(self, "_h", None):
            load().h2d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        s = h2d_stats()
        _check(load().h2d_info(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in h2d_stats._fields_ if f != "pad"}

    @property
    def n(self):
        return self.info()["n"]

    def matvec(self, x, prec="fp64", out=None):
        """y = A_hat x.  x: (N,) or (nrhs, N) float64 on the GPU (row r is RHS r)."""
        x = x.contiguous()
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        n = x.shape[-1]
        y = torch.empty_like(x) if out is None else out
        _check(load().h2d_matvec(self._h, _dev_f64(x, "x"), _dev_f64(y, "y"), nrhs, n, PREC[prec], _stream()))
        return y

    def matvec_noalloc(self, x, prec="fp64", out=None):
        """y = A_hat x (one right-hand side) on the library's fixed work array."""
        x = x.contiguous()
        y = torch.empty_like(x) if out is None else out
        _check(load().h2d_matvec_noalloc(self._h, _dev_f64(x, "x"), _dev_f64(y, "y"), PREC[prec], _stream()))
        return y

    def bj_setup(self):
        _check(load().h2d_bj_setup(self._h, _stream()))

    def precond_apply(self, r, precond="bj"):
        r = r.contiguous()
        z = torch.empty_like(r)
        _check(load().h2d_precond_apply(self._h, PRECOND[precond], _dev_f64(r, "r"), _dev_f64(z, "z"), _stream()))
        return z

    def solve(self, b, tol=1e-8, restart=50, max_iter=2500, mode="plain", inner_prec="fp16", inner_tol=1e-4,
              max_outer=50, precond="none"):
        b = b.contiguous()
        x = torch.empty_like(b)
        o = h2d_solve_opts(SOLVE_PLAIN if mode == "plain" else SOLVE_REFINE, int(restart), int(max_iter),
                           PREC[inner_prec], float(inner_tol), int(max_outer), PRECOND[precond])
        info = h2d_solve_info()
        st = load().h2d_solve(self._h, _dev_f64(b, "b"), _dev_f64(x, "x"), float(tol), C.byref(o), C.byref(info),
                              _stream())
        if st not in (H2D_OK, H2D_ENOCONV):
            _check(st)
        return x, {"iters": info.iters, "outer": info.outer, "relres": info.relres, "seconds": info.seconds,
                   "converged": st == H2D_OK, "fallback_at": info.fallback_at}

    def profile_enable(self, on=True):
        _check(load().h2d_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        """Average ms and algorithmic bytes per matvec kernel since the last read."""
        p = h2d_profile()
        _check(load().h2d_profile_read(self._h, C.byref(p)))
        return {"count": p.count, "prec": p.prec,
                "ms": dict(zip(PHASES, list(p.ms))), "bytes": dict(zip(PHASES, list(p.bytes)))}

    def mlp_train(self, n_solves=16, steps=1500, batch=4096, lr=5e-4, seed=1234, solve_tol=1e-10,
                  target="leaf", input="leaf") -> dict:
        o = h2d_mlp_train_opts(int(n_solves), int(steps), int(batch), float(lr), int(seed), float(solve_tol),
                               {"leaf": 0, "global": 1, "patch": 2}[target], {"leaf": 0, "patch": 1}[input])
        info = h2d_mlp_train_info()
        _check(load().h2d_mlp_train(self._h, C.byref(o), C.byref(info), _stream()))
        return {f: getattr(info, f) for f, _ in h2d_mlp_train_info._fields_}

    def mlp_weights(self, set_to=None, scale=None, patch=False):
        """Return (weights float32, scale); set them first if given.  patch:
        the handle's network was trained with the patch input (its weights
        are MLP_PARAMS_PATCH floats)."""
        import numpy as np
        size = MLP_PARAMS_PATCH if patch else MLP_PARAMS
        inp = None
        if set_to is not None:
            inp = np.ascontiguousarray(set_to, dtype=np.float32)
            assert inp.size == MLP_PARAMS
        sc = C.c_double(1.0 if scale is None else float(scale))
        if inp is not None:
            _check(load().h2d_mlp_weights(self._h, None, C.c_void_p(inp.ctypes.data), C.byref(sc), _stream()))
        out = np.empty(size, np.float32)
        _check(load().h2d_mlp_weights(self._h, C.c_void_p(out.ctypes.data), None, C.byref(sc), _stream()))
        return out, sc.value

    def autotune(self, nrhs=16):
        """Returns (picks, {(knob, candidate): ms}); picks = {knob: rows}."""
        chosen = (C.c_int32 * 3)()
        ms = (C.c_float * 9)()
        _check(load().h2d_autotune(self._h, int(nrhs), _stream(), chosen, ms))
        if nrhs > 1:
            return {"mr_rows": chosen[0]}, {("mr_rows", c): ms[i] for i, c in enumerate((128, 256, 512))}
        times = {("a_rows", c): ms[i] for i, c in enumerate((128, 256, 512))}
        times.update({("b1_rows", c): ms[3 + i] for i, c in enumerate((16, 32, 64))})
        times.update({("b2_rows", c): ms[6 + i] for i, c in enumerate((16, 32, 64))})
        return {"a_rows": chosen[0], "b1_rows": chosen[1], "b2_rows": chosen[2]}, times

    def set_item_rows(self, which, rows):
        """which: "a_rows" (single-RHS phase A), "mr_rows" (multi-RHS phase A),
        "b1_rows" (single-RHS phase B1) or "b2_rows" (single-RHS phase B2)."""
        w = {"a_rows": 0, "mr_rows": 1, "b1_rows": 2, "b2_rows": 3}[which]
        _check(load().h2d_set_item_rows(self._h, w, int(rows), _stream()))

    def export(self, path, factors=True):
        _check(load().h2d_export(self._h, str(path).encode(), 1 if factors else 0))


def mlp_loss_grad(W, X, T, M):
    """One MLP forward + backward on device FP32 tensors; returns (loss, grad)."""
    for t, nm in ((W, "W"), (X, "X"), (T, "T"), (M, "M")):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError(f"{nm} must be a contiguous float32 device tensor")
    g = torch.empty_like(W)
    loss = C.c_float()
    _check(load().h2d_mlp_loss_grad(C.c_void_p(W.data_ptr()), C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                    C.c_void_p(M.data_ptr()), int(X.shape[0]), C.byref(loss),
                                    C.c_void_p(g.data_ptr()), _stream()))
    return float(loss.value), g


class Batch:
    """Products of several handles captured into one HIP graph.

    xs[i], ys[i]: (nrhs, N_i) float64 device tensors bound at creation."""

    def __init__(self, handles, xs, ys):
        n = len(handles)
        nrhs = 1 if xs[0].dim() == 1 else xs[0].shape[0]
        P = C.c_void_p
        hs = (P * n)(*[h._h for h in handles])
        xp = (P * n)(*[_dev_f64(x, "x") for x in xs])
        yp = (P * n)(*[_dev_f64(y, "y") for y in ys])
        ld = (C.c_int64 * n)(*[x.shape[-1] for x in xs])
        self._b = P()
        self._keep = (handles, xs, ys)
        _check(load().h2d_batch_create(hs, n, nrhs, xp, yp, ld, C.byref(self._b)))

    def launch(self):
        _check(load().h2d_batch_launch(self._b, _stream()))

    def close(self):
        if getattr(self, "_b", None):
            load().h2d_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
