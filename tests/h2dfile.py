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
    assert version in (1, 2)
    adaptive = version == 2   # blocks carry the levels of both boxes
    fac = bool(flags & 1)
    H = {"factors": fac, "adaptive": adaptive}
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
    kap = H["kappa"]
    nn = int(take("<i8")[0])
    nt, ns, nD, ntl, nsl = [], [], [], [], []
    for _ in range(nn):
        tl, sl = map(int, take("<i4", 2)) if adaptive else (kap, kap)
        t, s = take("<i8", 2)
        nt.append(int(t)); ns.append(int(s)); ntl.append(tl); nsl.append(sl)
        if fac:
            m, c = int(levels[tl]["count"][t]), int(levels[sl]["count"][s])
            nD.append(take("<f8", m * c).reshape(c, m).T)
    H["near_tgt"] = np.array(nt, np.int64); H["near_src"] = np.array(ns, np.int64); H["near_D"] = nD
    H["near_tlevel"] = np.array(ntl, np.int32); H["near_slevel"] = np.array(nsl, np.int32)
    nb = int(take("<i8")[0])
    lv, kd, tg, sr, rk, fa, slv = [], [], [], [], [], [], []
    for _ in range(nb):
        l, k = map(int, take("<i4", 2))
        sl = int(take("<i4", 2)[0]) if adaptive else l
        t, s, r = map(int, take("<i8", 3))
        lv.append(l); kd.append(k); tg.append(t); sr.append(s); rk.append(r); slv.append(sl)
        if fac:
            m, c = int(levels[l]["count"][t]), int(levels[sl]["count"][s])
            if k == 1:
                fa.append(("D", take("<f8", m * c).reshape(c, m).T))
            else:
                U = take("<f8", m * r).reshape(r, m).T
                V = take("<f8", c * r).reshape(r, c).T
                fa.append(("UV", U, V))
    H["il_level"] = np.array(lv, np.int32); H["il_kind"] = np.array(kd, np.int32)
    H["il_tgt"] = np.array(tg, np.int64); H["il_src"] = np.array(sr, np.int64)
    H["il_rank"] = np.array(rk, np.int64); H["il_factors"] = fa
    H["il_slevel"] = np.array(slv, np.int32)
    assert off == len(buf), "trailing bytes"
    return H


def dense_operator(H):
    """The dense matrix the stored representation applies (caller order)."""
    n = H["n"]
    A = np.zeros((n, n))
    perm = H["perm"]
    lev = H["levels"]
    for tl, sl, t, s, D in zip(H["near_tlevel"], H["near_slevel"], H["near_tgt"], H["near_src"], H["near_D"]):
        r = perm[lev[tl]["begin"][t]:lev[tl]["begin"][t] + lev[tl]["count"][t]]
        c = perm[lev[sl]["begin"][s]:lev[sl]["begin"][s] + lev[sl]["count"][s]]
        A[np.ix_(r, c)] += D
    for l, sl, t, s, f in zip(H["il_level"], H["il_slevel"], H["il_tgt"], H["il_src"], H["il_factors"]):
        r = perm[lev[l]["begin"][t]:lev[l]["begin"][t] + lev[l]["count"][t]]
        c = perm[lev[sl]["begin"][s]:lev[sl]["begin"][s] + lev[sl]["count"][s]]
        A[np.ix_(r, c)] += f[1] if f[0] == "D" else f[1] @ f[2].T
    return A
