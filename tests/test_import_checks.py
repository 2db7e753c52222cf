"""h2d_import checks the whole file on the host before any upload: a file
whose permutation or level tables are inconsistent is refused with
H2D_EINVAL instead of driving out-of-range gathers on the device.  The
checks run before the first HIP call, so this test needs no GPU."""
import ctypes as C

import numpy as np
import pytest

from paper_2204_05536_amd import inputs

HEADER = 72          # magic, version, flags, pad, n, kappa, leaf, R, tol, kind, diag, c, diag_value


def _oracle_file(orc, tmp_path):
    xy, b, kern, leaf, tol = inputs.workload("log4096", n=300)
    O = orc.OracleH(xy, kern, 16, tol)
    p = tmp_path / "ok.h2dx"
    O.export(p)
    return p, xy.shape[0], O.kappa


def _level_offsets(buf, n, kappa):
    """Byte offsets of (nbox, key, begin, count, parent) of every level."""
    off = HEADER + 16 * n + 8 * n
    out = []
    for _ in range(kappa + 1):
        nb = int(np.frombuffer(buf, "<i8", 1, off)[0])
        key = off + 8
        begin = key + 4 * nb
        count = begin + 8 * nb
        parent = count + 8 * nb
        out.append((nb, key, begin, count, parent))
        off = parent + 8 * nb
    return out


def _import(path):
    from paper_2204_05536_amd import hodlr2d
    L = hodlr2d.load()
    out = C.c_void_p()
    st = L.h2d_import(str(path).encode(), 0, None, C.byref(out))
    msg = L.h2d_last_error().decode()
    return st, msg


def _poke(buf, off, dtype, value):
    b = bytearray(buf)
    b[off:off + np.dtype(dtype).itemsize] = np.array([value], dtype).tobytes()
    return bytes(b)


@pytest.mark.parametrize("what", ["perm_dup", "perm_range", "count_zero", "begin_gap", "parent_range",
                                  "parent_key", "key_order", "truncated"])
def test_corrupt_file_is_refused(orc, tmp_path, what):
    from paper_2204_05536_amd import hodlr2d
    p, n, kappa = _oracle_file(orc, tmp_path)
    buf = p.read_bytes()
    lv = _level_offsets(buf, n, kappa)
    perm0 = HEADER + 16 * n
    nb, key, begin, count, parent = lv[kappa]
    if what == "perm_dup":
        first = int(np.frombuffer(buf, "<i8", 1, perm0)[0])
        bad = _poke(buf, perm0 + 8, "<i8", first)
    elif what == "perm_range":
        bad = _poke(buf, perm0 + 8 * 5, "<i8", n)
    elif what == "count_zero":
        bad = _poke(buf, count + 8, "<i8", 0)
    elif what == "begin_gap":
        b1 = int(np.frombuffer(buf, "<i8", 1, begin + 8)[0])
        bad = _poke(buf, begin + 8, "<i8", b1 + 1)
    elif what == "parent_range":
        bad = _poke(buf, parent + 8 * (nb - 1), "<i8", lv[kappa - 1][0])
    elif what == "parent_key":
        # the last box's parent set to the first box of the level above
        # (a different key unless that level has one box)
        assert lv[kappa - 1][0] > 1
        bad = _poke(buf, parent + 8 * (nb - 1), "<i8", 0)
    elif what == "key_order":
        k0 = int(np.frombuffer(buf, "<u4", 1, key)[0])
        bad = _poke(buf, key + 4, "<u4", k0)
    else:
        bad = buf[: len(buf) // 2]
    q = tmp_path / "bad.h2dx"
    q.write_bytes(bad)
    st, msg = _import(q)
    assert st == hodlr2d.H2D_EINVAL, (what, st, msg)
