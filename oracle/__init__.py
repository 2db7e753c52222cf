"""HODLR2D CPU oracle (plain FP64 C, loaded through ctypes).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it to check the GPU library.  The library never imports
or links anything under ``oracle/``, and this package never imports the
library.

``build()`` compiles ``h2d_oracle.c`` with gcc into ``liboracle.so`` next to
this file.  ``OracleH`` runs Algorithm 1 (tree, lists, ACA) and exposes the
structure, the factors, Algorithm 2 and restarted GMRES.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "h2d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KINDS = {"log": 0, "invr": 1, "mq": 2, "gauss": 3, "phi1": 4, "phi2": 5, "sep": 6}
DIAG = {"replace": 0, "add": 1, "formula": 2}
BK_LOWRANK, BK_DENSE = 0, 1
ORC_OK, ORC_EINVAL, ORC_ENOMEM, ORC_EDUP, ORC_ENOCONV, ORC_EDEPTH = 0, 1, 2, 4, 5, 7


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (always, when force)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("diag_mode", C.c_int32), ("c", C.c_double),
                ("diag_value", C.c_double)]


def kernel_struct(spec: dict) -> _Kernel:
    return _Kernel(KINDS[spec["kind"]], DIAG[spec.get("diag_mode", "formula")],
                   float(spec.get("c", 0.0)), float(spec.get("diag_value", 0.0)))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        L.orc_build.argtypes = [dp, C.c_int64, C.POINTER(_Kernel), C.c_int32, C.c_double, C.c_int32,
                                C.POINTER(P)]
        L.orc_build.restype = C.c_int
        L.orc_free.argtypes = [P]
        L.orc_kappa.argtypes = [P]; L.orc_kappa.restype = C.c_int32
        L.orc_R.argtypes = [P]; L.orc_R.restype = C.c_double
        L.orc_perm.argtypes = [P, i64p]
        L.orc_nbox.argtypes = [P, C.c_int32]; L.orc_nbox.restype = C.c_int64
        L.orc_level.argtypes = [P, C.c_int32, C.POINTER(C.c_uint32), i64p, i64p, i64p]
        L.orc_n_near.argtypes = [P]; L.orc_n_near.restype = C.c_int64
        L.orc_n_il.argtypes = [P]; L.orc_n_il.restype = C.c_int64
        L.orc_near_table.argtypes = [P, i64p, i64p]
        L.orc_il_table.argtypes = [P, C.POINTER(C.c_int32), i64p, i64p, C.POINTER(C.c_int32), i64p]
        L.orc_il_factors.argtypes = [P, C.c_int64, dp, dp, dp]
        i32p = C.POINTER(C.c_int32)
        L.orc_is_adaptive.argtypes = [P]; L.orc_is_adaptive.restype = C.c_int32
        L.orc_is_symmetric.argtypes = [P]; L.orc_is_symmetric.restype = C.c_int32
        L.orc_block_levels.argtypes = [P, i32p, i32p, i32p, i32p]
        L.orc_admissible.argtypes = [C.c_int, C.c_uint32, C.c_int, C.c_uint32]
        L.orc_admissible.restype = C.c_int
        L.orc_near_factor.argtypes = [P, C.c_int64, dp]
        L.orc_matvec.argtypes = [P, dp, dp]; L.orc_matvec.restype = C.c_int
        L.orc_gmres.argtypes = [P, dp, dp, C.c_double, C.c_int32, C.c_int32, C.POINTER(C.c_int32), dp]
        L.orc_gmres.restype = C.c_int
        L.orc_export.argtypes = [P, C.c_char_p]; L.orc_export.restype = C.c_int
        L.orc_entry.argtypes = [C.POINTER(_Kernel), dp, C.c_int64, C.c_int64]
        L.orc_entry.restype = C.c_double
        L.orc_entries.argtypes = [C.POINTER(_Kernel), dp, i64p, i64p, C.c_int64, dp]
        L.orc_dense_rows.argtypes = [C.POINTER(_Kernel), dp, C.c_int64, i64p, C.c_int64, dp, dp]
        L.orc_box_radius.argtypes = [dp, C.c_int64]; L.orc_box_radius.restype = C.c_double
        L.orc_paper_id.argtypes = [C.c_uint32, C.c_uint32, C.c_int]; L.orc_paper_id.restype = C.c_uint32
        L.orc_morton_key.argtypes = [C.c_uint32, C.c_uint32, C.c_int]; L.orc_morton_key.restype = C.c_uint32
        L.orc_interaction_list.argtypes = [C.c_uint32, C.c_int, C.POINTER(C.c_uint32)]
        L.orc_interaction_list.restype = C.c_int
        L.orc_edge_list.argtypes = [C.c_uint32, C.c_int, C.POINTER(C.c_uint32)]
        L.orc_edge_list.restype = C.c_int
        L.orc_box_relation.argtypes = [C.c_uint32, C.c_uint32, C.c_int]
        L.orc_box_relation.restype = C.c_int
        L.orc_aca.argtypes = [C.POINTER(_Kernel), dp, i64p, C.c_int64, i64p, C.c_int64, C.c_double,
                              C.POINTER(C.c_int32), C.POINTER(dp), C.POINTER(dp), C.POINTER(dp)]
        L.orc_aca.restype = C.c_int64
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i64p(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def entries(spec, xy, I, J):
    """K(x_I[t], x_J[t]) for index arrays I, J (caller numbering)."""
    xy = _f64(xy); I = np.ascontiguousarray(I, np.int64); J = np.ascontiguousarray(J, np.int64)
    out = np.empty(I.shape[0])
    k = kernel_struct(spec)
    lib().orc_entries(C.byref(k), _dp(xy), _i64p(I), _i64p(J), I.shape[0], _dp(out))
    return out


def dense_matrix(spec, xy):
    """The full N x N kernel matrix by its definition (small N only)."""
    n = xy.shape[0]
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return entries(spec, xy, I.ravel(), J.ravel()).reshape(n, n)


def dense_rows(spec, xy, x, rows=None):
    """Rows of A x by the O(N) definition per row (rows=None: all)."""
    xy = _f64(xy); x = _f64(x)
    n = xy.shape[0]
    k = kernel_struct(spec)
    if rows is None:
        y = np.empty(n)
        lib().orc_dense_rows(C.byref(k), _dp(xy), n, None, n, _dp(x), _dp(y))
        return y
    rows = np.ascontiguousarray(rows, np.int64)
    y = np.empty(rows.shape[0])
    lib().orc_dense_rows(C.byref(k), _dp(xy), n, _i64p(rows), rows.shape[0], _dp(x), _dp(y))
    return y


def box_radius(xy):
    xy = _f64(xy)
    return lib().orc_box_radius(_dp(xy), xy.shape[0])


def paper_id(ix, iy, level):
    return int(lib().orc_paper_id(ix, iy, level))


def morton_key(ix, iy, level):
    return int(lib().orc_morton_key(ix, iy, level))


def interaction_list(key, level):
    out = (C.c_uint32 * 24)()
    c = lib().orc_interaction_list(key, level, out)
    return [int(out[i]) for i in range(c)]


def edge_list(key, level):
    out = (C.c_uint32 * 8)()
    c = lib().orc_edge_list(key, level, out)
    return [int(out[i]) for i in range(c)]


def box_relation(ka, kb, level):
    return int(lib().orc_box_relation(ka, kb, level))


def admissible(la, ka, lb, kb):
    """1 when boxes (level la, key ka) and (lb, kb) share at most one point."""
    return int(lib().orc_admissible(la, ka, lb, kb))


def aca(spec, xy, rows, cols, tol):
    """ACA of the block K(xy[rows], xy[cols]); returns (kind, rank, U, V, D)."""
    xy = _f64(xy)
    rows = np.ascontiguousarray(rows, np.int64); cols = np.ascontiguousarray(cols, np.int64)
    k = kernel_struct(spec)
    kind = C.c_int32()
    U = C.POINTER(C.c_double)(); V = C.POINTER(C.c_double)(); D = C.POINTER(C.c_double)()
    m, n = rows.shape[0], cols.shape[0]
    r = lib().orc_aca(C.byref(k), _dp(xy), _i64p(rows), m, _i64p(cols), n, tol,
                      C.byref(kind), C.byref(U), C.byref(V), C.byref(D))
    libc = C.CDLL(None)
    libc.free.argtypes = [C.c_void_p]
    if kind.value == BK_DENSE:
        Dm = np.ctypeslib.as_array(D, shape=(n * m,)).copy().reshape(n, m).T
        libc.free(C.cast(D, C.c_void_p))
        return BK_DENSE, int(r), None, None, Dm
    if r > 0:
        Um = np.ctypeslib.as_array(U, shape=(r * m,)).copy().reshape(r, m).T
        Vm = np.ctypeslib.as_array(V, shape=(r * n,)).copy().reshape(r, n).T
    else:
        Um = np.zeros((m, 0)); Vm = np.zeros((n, 0))
    libc.free(C.cast(U, C.c_void_p)); libc.free(C.cast(V, C.c_void_p))
    return BK_LOWRANK, int(r), Um, Vm, None


class OracleH:
    """Algorithm 1 on the CPU: the HODLR2D representation of K(xy, xy).

    ``factors=False`` builds the tree and the lists only (no ACA).
    ``adaptive=True`` builds the adaptive tree (a box is split exactly when
    it holds more than leaf_max points) and its blocks between boxes of any
    levels.
    ``symmetric=True`` (symmetric kernels, balanced tree) compresses only the
    block of each interaction-list pair whose target box has the smaller
    index; the mirror block is its exact transpose.
    """

    def __init__(self, xy, spec, leaf_max=64, tol=1e-10, factors=True, adaptive=False, symmetric=False):
        self.xy = _f64(xy)
        self.n = self.xy.shape[0]
        self.spec = dict(spec)
        self._k = kernel_struct(spec)
        h = C.c_void_p()
        st = lib().orc_build(_dp(self.xy), self.n, C.byref(self._k), int(leaf_max), float(tol),
                             (1 if factors else 0) | (2 if adaptive else 0) | (4 if symmetric else 0),
                             C.byref(h))
        if st != ORC_OK:
            raise OracleError(st, "build")
        self._h = h
        self.factors = factors
        self.leaf_max = leaf_max
        self.tol = tol

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    @property
    def kappa(self):
        return int(lib().orc_kappa(self._h))

    @property
    def R(self):
        return float(lib().orc_R(self._h))

    def perm(self):
        p = np.empty(self.n, np.int64)
        lib().orc_perm(self._h, _i64p(p))
        return p

    def level(self, l):
        nb = lib().orc_nbox(self._h, l)
        key = np.empty(nb, np.uint32); b = np.empty(nb, np.int64)
        c = np.empty(nb, np.int64); p = np.empty(nb, np.int64)
        lib().orc_level(self._h, l, key.ctypes.data_as(C.POINTER(C.c_uint32)), _i64p(b), _i64p(c), _i64p(p))
        return {"key": key, "begin": b, "count": c, "parent": p}

    def near_table(self):
        nn = lib().orc_n_near(self._h)
        t = np.empty(nn, np.int64); s = np.empty(nn, np.int64)
        lib().orc_near_table(self._h, _i64p(t), _i64p(s))
        return t, s

    def il_table(self):
        nb = lib().orc_n_il(self._h)
        lv = np.empty(nb, np.int32); t = np.empty(nb, np.int64); s = np.empty(nb, np.int64)
        kd = np.empty(nb, np.int32); rk = np.empty(nb, np.int64)
        lib().orc_il_table(self._h, lv.ctypes.data_as(C.POINTER(C.c_int32)), _i64p(t), _i64p(s),
                           kd.ctypes.data_as(C.POINTER(C.c_int32)), _i64p(rk))
        return {"level": lv, "tgt": t, "src": s, "kind": kd, "rank": rk}

    @property
    def adaptive(self):
        return bool(lib().orc_is_adaptive(self._h))

    @property
    def symmetric(self):
        return bool(lib().orc_is_symmetric(self._h))

    def block_levels(self):
        """(near target levels, near source levels, IL target levels, IL source levels)."""
        nn = lib().orc_n_near(self._h); ni = lib().orc_n_il(self._h)
        a = [np.empty(max(c, 1), np.int32) for c in (nn, nn, ni, ni)]
        lib().orc_block_levels(self._h, *[x.ctypes.data_as(C.POINTER(C.c_int32)) for x in a])
        return a[0][:nn], a[1][:nn], a[2][:ni], a[3][:ni]

    def il_factors(self, b):
        """(kind, U, V, D) of interaction-list block b, in tree-ordered rows/cols."""
        tab = self.il_table() if not hasattr(self, "_tab") else self._tab
        self._tab = tab
        if not hasattr(self, "_lv"):
            self._lv = self.block_levels()
        lt = self.level(int(tab["level"][b])); ls = self.level(int(self._lv[3][b]))
        m = int(lt["count"][tab["tgt"][b]]); n = int(ls["count"][tab["src"][b]])
        k = int(tab["rank"][b])
        if tab["kind"][b] == BK_DENSE:
            D = np.empty(m * n)
            lib().orc_il_factors(self._h, b, None, None, _dp(D))
            return BK_DENSE, None, None, D.reshape(n, m).T
        U = np.empty(max(m * k, 1)); V = np.empty(max(n * k, 1))
        lib().orc_il_factors(self._h, b, _dp(U), _dp(V), None)
        return BK_LOWRANK, U[:m * k].reshape(k, m).T, V[:n * k].reshape(k, n).T, None

    def near_factor(self, b):
        t, s = self.near_table()
        ntl, nsl, _, _ = self.block_levels()
        m = int(self.level(int(ntl[b]))["count"][t[b]]); n = int(self.level(int(nsl[b]))["count"][s[b]])
        D = np.empty(m * n)
        lib().orc_near_factor(self._h, b, _dp(D))
        return D.reshape(n, m).T

    def matvec(self, x):
        x = _f64(x)
        y = np.empty(self.n)
        st = lib().orc_matvec(self._h, _dp(x), _dp(y))
        if st != ORC_OK:
            raise OracleError(st, "matvec")
        return y

    def gmres(self, b, tol=1e-8, restart=50, max_iter=2500):
        b = _f64(b)
        x = np.empty(self.n)
        it = C.c_int32(); rr = C.c_double()
        st = lib().orc_gmres(self._h, _dp(b), _dp(x), tol, restart, max_iter, C.byref(it), C.byref(rr))
        return x, int(it.value), float(rr.value), st

    def export(self, path):
        st = lib().orc_export(self._h, str(path).encode())
        if st != ORC_OK:
            raise OracleError(st, "export")

    def dense(self):
        return dense_matrix(self.spec, self.xy)
