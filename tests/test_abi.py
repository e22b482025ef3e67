"""C ABI checks that need no GPU: exported symbols and descriptor validation."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "tmm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(tmm_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported():
    from paper_1410_0204_amd import tmm
    lib = tmm.load()
    names = _declared()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(tmm.EXPORTED) == names


def _desc(inp, **over):
    from paper_1410_0204_amd import tmm
    a = inp.desc_arrays()
    a.update({k: v for k, v in over.items()})
    keep = {k: (np.ascontiguousarray(v, dtype=np.int32) if np.asarray(v).dtype.kind in "iu"
                else np.ascontiguousarray(v, dtype=np.float64))
            for k, v in a.items() if isinstance(v, np.ndarray)}
    ip = lambda x: x.ctypes.data_as(C.POINTER(C.c_int))  # noqa: E731
    dp = lambda x: x.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    d = tmm.TmmDesc(a["n"], a["ncol"], a["nlayer"], ip(keep["col_start"]), dp(keep["lat"]), dp(keep["area"]),
                    dp(keep["dz"]), a["nmat"], a["nstep"], a["model"], a["neuphotic"], a.get("nbgc", 1),
                    over.get("nbatch_max", 1),
                    over.get("adjoint_nbatch_max", 1), over.get("ckpt_every", 240),
                    keep["ae_colidx"].size, ip(keep["ae_rowptr"]), ip(keep["ae_colidx"]), dp(keep["ae_val"]),
                    keep["ai_colidx"].size, ip(keep["ai_rowptr"]), ip(keep["ai_colidx"]), dp(keep["ai_val"]))
    return d, keep


def _status(d):
    from paper_1410_0204_amd import tmm
    n = C.c_size_t()
    return tmm.load().tmm_workspace_bytes(C.byref(d), C.byref(n)), n.value


def test_valid_descriptor_sizes_workspace(tiny_n):
    d, _ = _desc(tiny_n)
    rc, n = _status(d)
    assert rc == 0 and n > 0


def test_invalid_descriptors_are_rejected(tiny_n):
    tm = tiny_n.tm
    bad_rowptr = tm.ae_rowptr.copy()
    bad_rowptr[5], bad_rowptr[6] = bad_rowptr[6], bad_rowptr[5] - 1      # not monotone
    bad_col = tm.ae_colidx.copy()
    bad_col[3] = tiny_n.n                                                 # out of range
    cross = tm.ai_colidx.copy()
    cross[0] = tiny_n.grid.col_start[1]                                   # couples two columns
    for over in ({"ae_rowptr": bad_rowptr}, {"ae_colidx": bad_col}, {"ai_colidx": cross},
                 {"nstep": 2876}, {"nmat": 7}, {"model": 4}, {"neuphotic": 0},
                 {"ckpt_every": 7}, {"nbatch_max": 0}, {"adjoint_nbatch_max": 2}, {"nbgc": -1}, {"nbgc": 17},
                 {"dz": np.r_[tiny_n.grid.dz[:-1], -1.0]}):
        d, _ = _desc(tiny_n, **over)
        rc, _ = _status(d)
        assert rc == -1, over


def test_internal_bgc_steps_in_descriptor(small_ndop):
    """0/1 = one evaluation; up to 16 internal steps; more than 4 euphotic layers only without them."""
    for nbgc in (0, 1, 8, 16):
        d, _ = _desc(small_ndop, nbgc=nbgc)
        assert _status(d)[0] == 0, nbgc
    d, _ = _desc(small_ndop, nbgc=8, neuphotic=5)
    assert _status(d)[0] == -6
    d, _ = _desc(small_ndop, nbgc=1, neuphotic=5)
    assert _status(d)[0] == 0


def test_po4_dop_phy_descriptor():
    """Three tracers are accepted, with and without internal BGC steps (up to 4 euphotic layers)."""
    import synth
    inp = synth.tiny(model=synth.MODEL_NDOPPHY)
    d, _ = _desc(inp)
    assert _status(d)[0] == 0
    d, _ = _desc(inp, nbgc=8)
    assert _status(d)[0] == 0
    small = synth.small_ndop(model=synth.MODEL_NDOPPHY)
    d, _ = _desc(small, nbgc=8, neuphotic=5)
    assert _status(d)[0] == -6


def test_rows_without_diagonal_widen_the_stencil_table(small_ndop):
    """Every row keeps a stencil slot that reads the row itself (the member-parallel kernel takes the
    row's own state from it): a row of the greatest length without its diagonal widens the ELL table
    by one slot, so the workspace grows; the same change in a shorter row does not."""
    tm = small_ndop.tm
    lens = np.diff(tm.ae_rowptr)
    d, keep = _desc(small_ndop)            # keep: the arrays the descriptor points into
    base = _status(d)
    assert base[0] == 0

    def without_diagonal(i):
        col = tm.ae_colidx.copy()
        e0, e1 = tm.ae_rowptr[i], tm.ae_rowptr[i + 1]
        row = set(col[e0:e1].tolist())
        assert i in row
        spare = next(c for c in range(small_ndop.n) if c not in row)
        col[e0 + list(col[e0:e1]).index(i)] = spare
        return col

    full = int(np.argmax(lens))
    short = int(np.argmin(lens))
    assert lens[short] < lens[full]
    d, keep = _desc(small_ndop, ae_colidx=without_diagonal(full))
    rc, n = _status(d)
    assert rc == 0 and n > base[1]
    d, keep = _desc(small_ndop, ae_colidx=without_diagonal(short))
    rc, n = _status(d)
    assert rc == 0 and n == base[1]


def test_strerror():
    from paper_1410_0204_amd import tmm
    assert tmm.tmm_strerror(0) == "ok"
    assert "invalid" in tmm.tmm_strerror(-1)
    assert tmm.tmm_strerror(12345) == "unknown status"
