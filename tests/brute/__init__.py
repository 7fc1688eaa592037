"""ctypes wrapper around brute.c: exhaustive enumeration of local alignments.

Test-only.  Independent of the oracle and of the GPU library (no shared code).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libbrute.so")
_lock = threading.Lock()
_lib = None
MAXL = 16


def _load():
    global _lib
    with _lock:
        if _lib is None:
            src = os.path.join(_HERE, "brute.c")
            if (not os.path.exists(_SO)) or os.path.getmtime(_SO) < os.path.getmtime(src):
                subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", _SO, src],
                               check=True)
            lib = ctypes.CDLL(_SO)
            p8 = ctypes.POINTER(ctypes.c_int8)
            lib.brute_align.argtypes = [p8, ctypes.c_int, p8, ctypes.c_int, p8, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_uint8),
                                        ctypes.POINTER(ctypes.c_int)]
            lib.brute_align.restype = ctypes.c_int
            lib.brute_sub.argtypes = [p8, ctypes.c_int, p8, ctypes.c_int, p8, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_uint8),
                                      ctypes.POINTER(ctypes.c_int)]
            lib.brute_sub.restype = ctypes.c_int
            _lib = lib
    return _lib


def _runs(ops):
    """Op codes (0 M, 1 I, 2 D) to [(len, op)] runs."""
    cig = []
    for op in ops:
        ch = "MID"[int(op)]
        if cig and cig[-1][1] == ch:
            cig[-1] = (cig[-1][0] + 1, ch)
        else:
            cig.append((1, ch))
    return cig


def enumerate_align(q, r, matrix, o, e):
    """Returns dict(score1, maxcol, end=(ie, je), begin=(ib, jb), cigar=[(len, op)])."""
    lib = _load()
    q = np.ascontiguousarray(q, dtype=np.int8)
    r = np.ascontiguousarray(r, dtype=np.int8)
    m = np.ascontiguousarray(matrix, dtype=np.int8)
    if len(q) > MAXL or len(r) > MAXL:
        raise ValueError("brute force is limited to short sequences")
    s1 = ctypes.c_int64()
    maxcol = np.zeros(MAXL, dtype=np.int64)
    ends = (ctypes.c_int * 2)()
    begins = (ctypes.c_int * 2)()
    ops = np.zeros(2 * MAXL + 2, dtype=np.uint8)
    nops = ctypes.c_int()
    p8 = ctypes.POINTER(ctypes.c_int8)
    rc = lib.brute_align(q.ctypes.data_as(p8), len(q), r.ctypes.data_as(p8), len(r),
                         m.ctypes.data_as(p8), int(m.shape[0]), int(o), int(e),
                         ctypes.byref(s1), maxcol.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         ends, begins, ops.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                         ctypes.byref(nops))
    if rc != 0:
        raise ValueError("brute_align rejected the inputs")
    cig = _runs(ops[:nops.value])
    return dict(score1=s1.value, maxcol=maxcol[:len(r)].copy(),
                end=(ends[0], ends[1]), begin=(begins[0], begins[1]), cigar=cig)


def enumerate_sub(q, r, matrix, o, e, je, s):
    """The alignment of score s ending in column je (see brute_sub).  Returns
    dict(end=(ie, je), begin=(ib, jb), cigar=[(len, op)]), end (-1, -1) when
    no alignment of score s ends in column je."""
    lib = _load()
    q = np.ascontiguousarray(q, dtype=np.int8)
    r = np.ascontiguousarray(r, dtype=np.int8)
    m = np.ascontiguousarray(matrix, dtype=np.int8)
    if len(q) > MAXL or len(r) > MAXL:
        raise ValueError("brute force is limited to short sequences")
    ends = (ctypes.c_int * 2)()
    begins = (ctypes.c_int * 2)()
    ops = np.zeros(2 * MAXL + 2, dtype=np.uint8)
    nops = ctypes.c_int()
    p8 = ctypes.POINTER(ctypes.c_int8)
    rc = lib.brute_sub(q.ctypes.data_as(p8), len(q), r.ctypes.data_as(p8), len(r),
                       m.ctypes.data_as(p8), int(m.shape[0]), int(o), int(e), int(je), int(s),
                       ends, begins, ops.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                       ctypes.byref(nops))
    if rc != 0:
        raise ValueError("brute_sub rejected its inputs")
    return {"end": (ends[0], ends[1]), "begin": (begins[0], begins[1]),
            "cigar": _runs(ops[:nops.value])}
