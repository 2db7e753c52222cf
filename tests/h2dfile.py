"""Reader of the "H2DX" version-1 file written by the oracle and by
h2d_export (format documented in include/h2d.h and the oracle source)."""
import numpy as np


def read(path):
    with open(path, "rb") as f:
        buf = f.read()
    off = 0

    def take(dtype, count=1):
        nonlocal off
        dt = np.dtype(dtype)
        a = np.frombuffer(buf, dtype=dt, count=count, offset=off)
        off += dt.itemsize * count
        return a

    assert buf[:4] == b"H2DX"
    off = 4
    version, flags, _ = take("<u4", 3)
    assert version == 1
    fac = bool(flags & 1)
    H = {"factors": fac}
    H["n"] = int(take("<i8")[0])
    H["kappa"] = int(take("<i4")[0])
    H["leaf_max"] = int(take("<i4")[0])
    H["R"], H["tol"] = map(float, take("<f8", 2))
    H["kind"], H["diag_mode"] = map(int, take("<i4", 2))
    H["c"], H["diag_value"] = map(float, take("<f8", 2))
    n = H["n"]
    H["xy"] = take("<f8", 2 * n).reshape(n, 2)
    H["perm"] = take("<i8", n).copy()
    levels = []
    for _ in range(H["kappa"] + 1):
        nb = int(take("<i8")[0])
        key = take("<u4", nb).copy()
        levels.append({"key": key, "begin": take("<i8", nb).copy(), "count": take("<i8", nb).copy(),
                       "parent": take("<i8", nb).copy()})
    H["levels"] = levels
    LL = levels[-1]
    nn = int(take("<i8")[0])
    nt, ns, nD = [], [], []
    for _ in range(nn):
        t, s = take("<i8", 2)
        nt.append(int(t)); ns.append(int(s))
        if fac:
            m, c = int(LL["count"][t]), int(LL["count"][s])
            nD.append(take("<f8", m * c).reshape(c, m).T)
    H["near_tgt"] = np.array(nt, np.int64); H["near_src"] = np.array(ns, np.int64); H["near_D"] = nD
    nb = int(take("<i8")[0])
    lv, kd, tg, sr, rk, fa = [], [], [], [], [], []
    for _ in range(nb):
        l, k = map(int, take("<i4", 2))
        t, s, r = map(int, take("<i8", 3))
        lv.append(l); kd.append(k); tg.append(t); sr.append(s); rk.append(r)
        if fac:
            L = levels[l]
            m, c = int(L["count"][t]), int(L["count"][s])
            if k == 1:
                fa.append(("D", take("<f8", m * c).reshape(c, m).T))
            else:
                U = take("<f8", m * r).reshape(r, m).T
                V = take("<f8", c * r).reshape(r, c).T
                fa.append(("UV", U, V))
    H["il_level"] = np.array(lv, np.int32); H["il_kind"] = np.array(kd, np.int32)
    H["il_tgt"] = np.array(tg, np.int64); H["il_src"] = np.array(sr, np.int64)
    H["il_rank"] = np.array(rk, np.int64); H["il_factors"] = fa
    assert off == len(buf), "trailing bytes"
    return H


def dense_operator(H):
    """The dense matrix the stored representation applies (caller order)."""
    n = H["n"]
    A = np.zeros((n, n))
    perm = H["perm"]
    LL = H["levels"][-1]
    for t, s, D in zip(H["near_tgt"], H["near_src"], H["near_D"]):
        r = perm[LL["begin"][t]:LL["begin"][t] + LL["count"][t]]
        c = perm[LL["begin"][s]:LL["begin"][s] + LL["count"][s]]
        A[np.ix_(r, c)] += D
    for l, t, s, f in zip(H["il_level"], H["il_tgt"], H["il_src"], H["il_factors"]):
        L = H["levels"][l]
        r = perm[L["begin"][t]:L["begin"][t] + L["count"][t]]
        c = perm[L["begin"][s]:L["begin"][s] + L["count"][s]]
        A[np.ix_(r, c)] += f[1] if f[0] == "D" else f[1] @ f[2].T
    return A
