"""Plain CPU reference (the oracle) for the SSW alignment path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
never imports, links or calls it, and the two share no code.

The arithmetic lives in ``sw_oracle.c`` (plain C, int64 scores, built with
``-O2 -fno-tree-vectorize``); this module only marshals arguments.  Each C
function cites the step of the paper's method section it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

FLAG_BEGIN = 1
FLAG_CIGAR = 2
FLAG_SCORE2 = 4
FLAG_ALL = 7


class _Res(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "score1", "score2", "read_begin1", "read_end1",
        "ref_begin1", "ref_end1", "ref_end2", "cigar_len")]


def build(force: bool = False) -> str:
    """Compile liboracle.so with make (gcc)."""
    if force or not os.path.exists(_LIB_PATH):
        subprocess.run(["make", "-s", "-C", _HERE, "-B" if force else "liboracle.so"],
                       check=True)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            p8 = ctypes.POINTER(ctypes.c_int8)
            p64 = ctypes.POINTER(ctypes.c_int64)
            pu32 = ctypes.POINTER(ctypes.c_uint32)
            i64, i32, u32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
            lib.orc_fill.argtypes = [p8, i64, p8, i64, p8, i32, i32, i32, p64, p64, p64, p64]
            lib.orc_fill.restype = None
            lib.orc_begin_reverse.argtypes = [p8, p8, p8, i32, i32, i32, i64, i64, i64, p64, p64]
            lib.orc_begin_reverse.restype = ctypes.c_int
            lib.orc_begin_startprop.argtypes = [p8, i64, p8, i64, p8, i32, i32, i32,
                                                i64, i64, i64, p64, p64]
            lib.orc_begin_startprop.restype = ctypes.c_int
            lib.orc_traceback.argtypes = [p8, p8, p8, i32, i32, i32, i64, i64, i64, i64,
                                          pu32, i64, p64]
            lib.orc_traceback.restype = ctypes.c_int64
            lib.orc_score2.argtypes = [p64, i64, i64, i64, i64, p64, p64]
            lib.orc_score2.restype = None
            lib.orc_align.argtypes = [p8, i64, p8, i64, p8, i32, i32, i32, u32, i64,
                                      ctypes.POINTER(_Res), pu32, i64, p64]
            lib.orc_align.restype = ctypes.c_int
            lib.orc_align_many.argtypes = [p8, p64, p8, p64, p64, p64, i64, p8, i32, i32, i32,
                                           u32, i64, ctypes.POINTER(_Res), pu32, p64, i32]
            lib.orc_align_many.restype = ctypes.c_int64
            lib.orc_column_row.argtypes = [p8, i64, p8, i64, p8, i32, i32, i32, i64, i64]
            lib.orc_column_row.restype = ctypes.c_int64
            lib.orc_suboptimal.argtypes = [p8, i64, p8, i64, p8, i32, i32, i32, i64, i64,
                                           ctypes.POINTER(_Sub), pu32, i64]
            lib.orc_suboptimal.restype = ctypes.c_int
            lib.orc_suboptimal_many.argtypes = [p8, p64, p8, p64, p64, p64, i64, p8, i32, i32,
                                                i32, p64, p64, ctypes.POINTER(_Sub), pu32, p64,
                                                i32]
            lib.orc_suboptimal_many.restype = ctypes.c_int64
            _lib = lib
    return _lib


def _i8(a):
    a = np.ascontiguousarray(a, dtype=np.int8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _mat(matrix):
    m = np.ascontiguousarray(matrix, dtype=np.int8)
    if m.ndim != 2 or m.shape[0] != m.shape[1]:
        raise ValueError("matrix must be square n x n")
    return m, int(m.shape[0])


@dataclass
class Alignment:
    score1: int
    score2: int
    read_begin1: int
    read_end1: int
    ref_begin1: int
    ref_end1: int
    ref_end2: int
    cigar: list = field(default_factory=list)   # list of (length, op) with op in "MID"

    def cigar_string(self) -> str:
        return "".join(f"{n}{op}" for n, op in self.cigar)


def decode_cigar(words) -> list:
    ops = "MID"
    return [(int(w) >> 4, ops[int(w) & 0xF]) for w in words]


def fill(q, r, matrix, o, e):
    """Forward pass: (score1, qend, rend, maxcol[int64])."""
    lib = _load()
    q, qp = _i8(q)
    r, rp = _i8(r)
    m, n = _mat(matrix)
    maxcol = np.zeros(max(len(r), 1), dtype=np.int64)
    s = ctypes.c_int64(); qe = ctypes.c_int64(); re_ = ctypes.c_int64()
    lib.orc_fill(qp, len(q), rp, len(r), m.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                 n, int(o), int(e), maxcol.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                 ctypes.byref(s), ctypes.byref(qe), ctypes.byref(re_))
    return s.value, qe.value, re_.value, maxcol[:len(r)]


def begin_reverse(q, r, matrix, o, e, qend, rend, score1):
    lib = _load()
    q, qp = _i8(q)
    r, rp = _i8(r)
    m, n = _mat(matrix)
    qb = ctypes.c_int64(); rb = ctypes.c_int64()
    rc = lib.orc_begin_reverse(qp, rp, m.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), n,
                               int(o), int(e), int(qend), int(rend), int(score1),
                               ctypes.byref(qb), ctypes.byref(rb))
    if rc != 0:
        raise RuntimeError("reversed pass did not reach score1")
    return qb.value, rb.value


def begin_startprop(q, r, matrix, o, e, qend, rend, score1):
    lib = _load()
    q, qp = _i8(q)
    r, rp = _i8(r)
    m, n = _mat(matrix)
    qb = ctypes.c_int64(); rb = ctypes.c_int64()
    rc = lib.orc_begin_startprop(qp, len(q), rp, len(r),
                                 m.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), n,
                                 int(o), int(e), int(qend), int(rend), int(score1),
                                 ctypes.byref(qb), ctypes.byref(rb))
    if rc != 0:
        raise RuntimeError("start propagation did not reach score1")
    return qb.value, rb.value


def traceback(q, r, matrix, o, e, qbeg, qend, rbeg, rend):
    """Global DP + traceback on the rectangle: (global_score, cigar words)."""
    lib = _load()
    q, qp = _i8(q)
    r, rp = _i8(r)
    m, n = _mat(matrix)
    cap = (qend - qbeg + 1) + (rend - rbeg + 1) + 1
    buf = np.zeros(max(cap, 1), dtype=np.uint32)
    gs = ctypes.c_int64()
    runs = lib.orc_traceback(qp, rp, m.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), n,
                             int(o), int(e), int(qbeg), int(qend), int(rbeg), int(rend),
                             buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), cap,
                             ctypes.byref(gs))
    if runs < 0:
        raise MemoryError("oracle traceback allocation failed")
    return gs.value, buf[:runs].copy()


def score2(maxcol, ref_begin1, ref_end1, mask_len):
    lib = _load()
    mc, mp = _i64(maxcol)
    s = ctypes.c_int64(); at = ctypes.c_int64()
    lib.orc_score2(mp, len(mc), int(ref_begin1), int(ref_end1), int(mask_len),
                   ctypes.byref(s), ctypes.byref(at))
    return s.value, at.value


def align(q, r, matrix, o, e, flags=FLAG_ALL, mask_len=-1, with_maxcol=False):
    """The whole path for one pair.  Returns an Alignment (and maxcol)."""
    lib = _load()
    q, qp = _i8(q)
    r, rp = _i8(r)
    m, n = _mat(matrix)
    cap = len(q) + len(r) + 1
    buf = np.zeros(cap, dtype=np.uint32)
    mc = np.zeros(max(len(r), 1), dtype=np.int64)
    res = _Res()
    rc = lib.orc_align(qp, len(q), rp, len(r), m.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                       n, int(o), int(e), int(flags), int(mask_len), ctypes.byref(res),
                       buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), cap,
                       mc.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise RuntimeError("oracle internal inconsistency")
    a = Alignment(res.score1, res.score2, res.read_begin1, res.read_end1,
                  res.ref_begin1, res.ref_end1, res.ref_end2,
                  decode_cigar(buf[:res.cigar_len]))
    return (a, mc[:len(r)]) if with_maxcol else a


def align_many(qcat, qoff, rcat, roff, pair_q, pair_r, matrix, o, e,
               flags=FLAG_ALL, mask_len=-1, nthreads=None):
    """Many pairs over threads.  Returns (records[npairs, 8] int64, cigar words,
    cigar offsets).  Record columns: score1, score2, read_begin1, read_end1,
    ref_begin1, ref_end1, ref_end2, cigar_len."""
    lib = _load()
    qcat, qcp = _i8(qcat)
    rcat, rcp = _i8(rcat)
    qoff, qop = _i64(qoff)
    roff, rop = _i64(roff)
    pq, pqp = _i64(pair_q)
    pr, prp = _i64(pair_r)
    m, n = _mat(matrix)
    npairs = len(pq)
    lens = (qoff[pq + 1] - qoff[pq]) + (roff[pr + 1] - roff[pr]) + 1
    coff = np.zeros(npairs + 1, dtype=np.int64)
    if npairs:
        coff[1:] = np.cumsum(lens)
    cig = np.zeros(max(int(coff[-1]), 1), dtype=np.uint32)
    res = (_Res * max(npairs, 1))()
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    fails = lib.orc_align_many(qcp, qop, rcp, rop, pqp, prp, npairs,
                               m.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), n,
                               int(o), int(e), int(flags), int(mask_len), res,
                               cig.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                               coff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               int(nthreads))
    if fails:
        raise RuntimeError(f"oracle failed on {fails} pairs")
    rec = np.frombuffer(res, dtype=np.int64).reshape(-1, 8)[:npairs].copy()
    return rec, cig, coff


class _Sub(ctypes.Structure):
    _fields_ = [("read_begin2", ctypes.c_int64), ("read_end2", ctypes.c_int64),
                ("ref_begin2", ctypes.c_int64), ("cigar_len", ctypes.c_int64)]


def column_row(q, r, matrix, o, e, col, target):
    """Smallest row i with H(i, col) == target, or -1."""
    lib = _load()
    q, qp = _i8(q)
    r, rp = _i8(r)
    m, n = _mat(matrix)
    return int(lib.orc_column_row(qp, len(q), rp, len(r),
                                  m.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), n, int(o),
                                  int(e), int(col), int(target)))


def suboptimal(q, r, matrix, o, e, score2, ref_end2):
    """The alignment behind score2: (read_begin2, read_end2, ref_begin2,
    [(len, op)]); all -1 and [] when score2 <= 0."""
    lib = _load()
    q, qp = _i8(q)
    r, rp = _i8(r)
    m, n = _mat(matrix)
    cap = len(q) + len(r) + 1
    buf = np.zeros(cap, dtype=np.uint32)
    res = _Sub()
    rc = lib.orc_suboptimal(qp, len(q), rp, len(r),
                            m.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), n, int(o), int(e),
                            int(score2), int(ref_end2), ctypes.byref(res),
                            buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), cap)
    if rc != 0:
        raise RuntimeError("oracle internal inconsistency (suboptimal)")
    return res.read_begin2, res.read_end2, res.ref_begin2, decode_cigar(buf[:res.cigar_len])


def suboptimal_many(qcat, qoff, rcat, roff, pair_q, pair_r, matrix, o, e, score2, ref_end2,
                    nthreads=None):
    """The suboptimal alignment of many pairs (score2, ref_end2 per pair from
    align_many).  Returns (records[npairs, 4] int64: read_begin2, read_end2,
    ref_begin2, cigar_len; cigar words; cigar offsets)."""
    lib = _load()
    qcat, qcp = _i8(qcat)
    rcat, rcp = _i8(rcat)
    qoff, qop = _i64(qoff)
    roff, rop = _i64(roff)
    pq, pqp = _i64(pair_q)
    pr, prp = _i64(pair_r)
    s2, s2p = _i64(score2)
    e2, e2p = _i64(ref_end2)
    m, n = _mat(matrix)
    npairs = len(pq)
    lens = (qoff[pq + 1] - qoff[pq]) + (roff[pr + 1] - roff[pr]) + 1
    coff = np.zeros(npairs + 1, dtype=np.int64)
    if npairs:
        coff[1:] = np.cumsum(lens)
    cig = np.zeros(max(int(coff[-1]), 1), dtype=np.uint32)
    res = (_Sub * max(npairs, 1))()
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    fails = lib.orc_suboptimal_many(qcp, qop, rcp, rop, pqp, prp, npairs,
                                    m.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), n, int(o),
                                    int(e), s2p, e2p, res,
                                    cig.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                    coff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    int(nthreads))
    if fails:
        raise RuntimeError(f"oracle failed on {fails} pairs (suboptimal)")
    rec = np.frombuffer(res, dtype=np.int64).reshape(-1, 4)[:npairs].copy()
    return rec, cig, coff
