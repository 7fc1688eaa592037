"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/swx.h, and rejects bad arguments before touching a GPU."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import paper_1208_6350_amd as swx
from paper_1208_6350_amd import _binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "swx.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(swx_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = swx.lib()
    names = _declared()
    assert "swx_align" in names and "swx_align_batch" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_binding.EXPORTED)


def test_strerror_and_codes():
    assert swx.swx_strerror(0) == "ok"
    assert swx.swx_strerror(-1) == "invalid argument"
    assert swx.swx_strerror(-99) == "unknown status"


def _profile_status(query, matrix, o, e, ctx=None):
    lib = swx.lib()
    q = np.ascontiguousarray(query, dtype=np.int8)
    m = np.ascontiguousarray(matrix, dtype=np.int8)
    h = ctypes.c_void_p()
    st = lib.swx_profile_create(ctx, q.ctypes.data if len(q) else None, len(q), m.ctypes.data,
                                int(m.shape[0]), o, e, ctypes.byref(h))
    return st, swx.swx_last_error()


def test_profile_argument_validation():
    dna = np.full((4, 4), -2, dtype=np.int8)
    np.fill_diagonal(dna, 2)
    assert _profile_status([0, 1], dna, 1, 3)[0] == -1            # o < e
    assert _profile_status([0, 1], dna, 3, -1)[0] == -1           # e < 0
    assert _profile_status([], dna, 3, 1)[0] == -1                # qlen < 1
    assert _profile_status([0, 4], dna, 3, 1)[0] == -1            # symbol >= n
    big = np.zeros((33, 33), dtype=np.int8)
    assert _profile_status([0], big, 3, 1)[0] == -1               # n > 32
    st, msg = _profile_status([0, 1], dna, 3, 1)                  # valid, but ctx is null
    assert st == -1 and "ctx" in msg


def test_null_pointers_rejected():
    lib = swx.lib()
    assert lib.swx_ctx_create(0, None) == -1
    assert lib.swx_align_batch(None, None, None, None) == -1
    assert lib.swx_align(None, None, 0, 0, -1, None, None) == -1
    assert lib.swx_graph_run(None, None) == -1
    assert lib.swx_profile_destroy(None) == -1
    lib.swx_result_free(None)   # no-op


def test_ctx_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = swx.lib().swx_ctx_create(0, ctypes.byref(h))
    assert st in (-3, -1) and h.value is None


def test_cigar_bound():
    qoff = np.array([0, 3, 5], dtype=np.int64)
    roff = np.array([0, 10], dtype=np.int64)
    dna = np.eye(4, dtype=np.int8)
    b = swx.swx_cigar_bound(dna, 3, 1, np.zeros(5, np.int8), qoff, np.zeros(10, np.int8), roff,
                            np.array([0, 1]), np.array([0, 0]))
    assert b == (3 + 10 + 1) + (2 + 10 + 1)
    assert swx.swx_cigar_bound(dna, 3, 1, np.zeros(5, np.int8), qoff, np.zeros(10, np.int8), roff,
                               np.array([2]), np.array([0])) == -1
