"""ctypes declarations of the C ABI in include/swx.h, plus a small Context
wrapper.  Argument marshalling only: no alignment arithmetic happens here."""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libswx.so"
_lock = threading.Lock()
_lib = None

SWX_OK = 0
SWX_BEGIN = 1
SWX_CIGAR = 2
SWX_SCORE2 = 4
SWX_ALL = 7
SWX_SUBOPT = 8
SWX_MEM_HOST = 0
SWX_MEM_DEVICE = 1
SWX_REF_DEVICE = 1 << 8
SWX_ERANGE = -6

REC_DTYPE = np.dtype([
    ("score1", "<i4"), ("score2", "<i4"), ("read_begin1", "<i4"), ("read_end1", "<i4"),
    ("ref_begin1", "<i8"), ("ref_end1", "<i8"), ("ref_end2", "<i8"), ("cigar_off", "<i8"),
    ("cigar_len", "<i4"), ("lane_bits", "<i4")])
assert REC_DTYPE.itemsize == 56


class SwxRec(ctypes.Structure):
    _fields_ = [("score1", ctypes.c_int32), ("score2", ctypes.c_int32),
                ("read_begin1", ctypes.c_int32), ("read_end1", ctypes.c_int32),
                ("ref_begin1", ctypes.c_int64), ("ref_end1", ctypes.c_int64),
                ("ref_end2", ctypes.c_int64), ("cigar_off", ctypes.c_int64),
                ("cigar_len", ctypes.c_int32), ("lane_bits", ctypes.c_int32)]


class SwxResult(ctypes.Structure):
    _fields_ = [("rec", SwxRec), ("cigar", ctypes.POINTER(ctypes.c_uint32)),
                ("sub", SwxRec), ("sub_cigar", ctypes.POINTER(ctypes.c_uint32))]


class SwxBatch(ctypes.Structure):
    _fields_ = [("matrix", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32),
                ("qcat", ctypes.c_void_p), ("qcat_len", ctypes.c_int64),
                ("qoff", ctypes.c_void_p), ("nq", ctypes.c_int64),
                ("rcat", ctypes.c_void_p), ("rcat_len", ctypes.c_int64),
                ("roff", ctypes.c_void_p), ("nr", ctypes.c_int64),
                ("pair_q", ctypes.c_void_p), ("pair_r", ctypes.c_void_p),
                ("npairs", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("mask_len", ctypes.c_int32), ("in_mem", ctypes.c_uint32)]


class SwxBatchOut(ctypes.Structure):
    _fields_ = [("recs", ctypes.c_void_p), ("cigar", ctypes.c_void_p),
                ("cigar_cap", ctypes.c_int64), ("cigar_used", ctypes.c_int64),
                ("out_mem", ctypes.c_uint32), ("pad_", ctypes.c_uint32),
                ("sub_recs", ctypes.c_void_p)]


class SwxTuning(ctypes.Structure):
    _fields_ = [("long_cells", ctypes.c_int64), ("long_rlen", ctypes.c_int64),
                ("intra_jobs", ctypes.c_int64), ("fill_rows", ctypes.c_int32),
                ("side_streams", ctypes.c_int32), ("fill_sched", ctypes.c_int32),
                ("fill_coop", ctypes.c_int32), ("intra_bits", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class SwxServerCfg(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("matrix", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32),
                ("mem_budget", ctypes.c_int64), ("max_pending", ctypes.c_int32),
                ("workers", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("mask_len", ctypes.c_int32),
                ("long_cells", ctypes.c_int64), ("graph_batch", ctypes.c_int32),
                ("graph_max_qlen", ctypes.c_int32), ("graph_max_rlen", ctypes.c_int64),
                ("side_streams", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class SwxServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("submitted", "deferred", "admitted", "completed", "batches", "max_batch_seen",
                 "graph_batches", "pending", "inflight_bytes", "peak_inflight_bytes")]


REQ_DTYPE = np.dtype([("query_id", "<i8"), ("query", "<u8"), ("qlen", "<i4"), ("_pad", "<i4"),
                      ("ref", "<u8"), ("rlen", "<i8"), ("tag", "<u8")])
assert REQ_DTYPE.itemsize == 48
COMPLETION_DTYPE = np.dtype([("ticket", "<u8"), ("tag", "<u8"), ("status", "<i4"),
                             ("batch_size", "<i4"), ("rec", REC_DTYPE), ("cigar", "<u8"),
                             ("t_submit_ns", "<i8"), ("t_start_ns", "<i8"), ("t_done_ns", "<i8")])
assert COMPLETION_DTYPE.itemsize == 112

class SwxGraphCfg(ctypes.Structure):
    _fields_ = [("matrix", ctypes.c_void_p), ("n", ctypes.c_int32), ("gap_open", ctypes.c_int32),
                ("gap_extend", ctypes.c_int32), ("max_pairs", ctypes.c_int64),
                ("max_qlen", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("max_rlen", ctypes.c_int64), ("qcat_cap", ctypes.c_int64),
                ("rcat_cap", ctypes.c_int64), ("nq_cap", ctypes.c_int64),
                ("nr_cap", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("mask_len", ctypes.c_int32), ("route", ctypes.c_int32), ("pad2_", ctypes.c_int32)]


class SwxGraphIo(ctypes.Structure):
    _fields_ = [("qcat", ctypes.c_void_p), ("qoff", ctypes.c_void_p), ("rcat", ctypes.c_void_p),
                ("roff", ctypes.c_void_p), ("pair_q", ctypes.c_void_p),
                ("pair_r", ctypes.c_void_p), ("recs", ctypes.c_void_p),
                ("cigar", ctypes.c_void_p), ("cigar_cap", ctypes.c_int64)]


class SwxSimModel(ctypes.Structure):
    _fields_ = [("cells_per_us", ctypes.c_double), ("batch_us", ctypes.c_double),
                ("request_us", ctypes.c_double)]


# name -> (restype, argtypes)
_SIGS = {
    "swx_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "swx_ctx_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "swx_profile_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "swx_profile_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "swx_align": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.c_uint32, ctypes.c_int32, ctypes.c_void_p,
                                 ctypes.POINTER(SwxResult)]),
    "swx_result_free": (None, [ctypes.POINTER(SwxResult)]),
    "swx_align_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SwxBatch),
                                       ctypes.POINTER(SwxBatchOut), ctypes.c_void_p]),
    "swx_align_batch_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SwxBatch),
                                               ctypes.POINTER(SwxBatchOut), ctypes.c_void_p]),
    "swx_cigar_bound": (ctypes.c_int64, [ctypes.POINTER(SwxBatch)]),
    "swx_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "swx_last_error": (ctypes.c_char_p, []),
    "swx_last_stage_ms": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.c_int]),
    "swx_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SwxTuning)]),
    "swx_graph_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SwxGraphCfg),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(SwxGraphIo)]),
    "swx_graph_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "swx_graph_run_eager": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "swx_graph_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SwxBatch)]),
    "swx_graph_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(SwxBatchOut)]),
    "swx_graph_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "swx_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SwxBatch), ctypes.c_int64,
                                    ctypes.c_char_p, ctypes.POINTER(SwxTuning),
                                    ctypes.POINTER(ctypes.c_int32)]),
    "swx_server_create": (ctypes.c_int, [ctypes.POINTER(SwxServerCfg),
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "swx_server_register_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_int64)]),
    "swx_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "swx_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "swx_completion_free": (None, [ctypes.c_void_p, ctypes.c_int32]),
    "swx_server_stats_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SwxServerStats)]),
    "swx_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "swx_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SwxTuning)]),
    "swx_check_max3": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(ctypes.c_uint64)]),
    "swx_lane_probe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_double)]),
    "swx_server_simulate": (ctypes.c_int, [ctypes.POINTER(SwxServerCfg), ctypes.POINTER(SwxSimModel),
                                           ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.POINTER(SwxServerStats)]),
}
EXPORTED = tuple(_SIGS)


def lib_path() -> str:
    return os.path.join(_HERE, _LIB_NAME)


def lib():
    """Load libswx.so (built in-tree by build.py).  Raises when it is missing."""
    global _lib
    with _lock:
        if _lib is None:
            path = lib_path()
            if not os.path.exists(path):
                raise RuntimeError(
                    f"{path} is missing: build it with `python -m paper_1208_6350_amd.build` "
                    "(there is no CPU fallback)")
            # One HIP runtime per process: torch carries its own libamdhip64
            # under the same soname as the system's, so it is loaded first and
            # the library binds to that copy (loaded the other way round,
            # torch finds no device).
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            L = ctypes.CDLL(path)
            for name, (res, args) in _SIGS.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


class SwxError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = lib().swx_last_error().decode(errors="replace")
        super().__init__(f"{where}: {lib().swx_strerror(status).decode()} ({status}): {detail}")


def _check(status: int, where: str):
    if status != SWX_OK:
        raise SwxError(status, where)


# ---- raw C entry points, same names as the header ---------------------------
def swx_ctx_create(device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(lib().swx_ctx_create(int(device), ctypes.byref(h)), "swx_ctx_create")
    return h.value


def swx_ctx_destroy(ctx: int) -> None:
    _check(lib().swx_ctx_destroy(ctx), "swx_ctx_destroy")


def swx_profile_create(ctx: int, query, matrix, gap_open: int, gap_extend: int) -> int:
    q = np.ascontiguousarray(query, dtype=np.int8)
    m = np.ascontiguousarray(matrix, dtype=np.int8)
    h = ctypes.c_void_p()
    _check(lib().swx_profile_create(ctx, q.ctypes.data, len(q), m.ctypes.data, int(m.shape[0]),
                                    int(gap_open), int(gap_extend), ctypes.byref(h)),
           "swx_profile_create")
    return h.value


def swx_profile_destroy(p: int) -> None:
    _check(lib().swx_profile_destroy(p), "swx_profile_destroy")


def decode_cigar(words) -> list:
    ops = "MID"
    return [(int(w) >> 4, ops[int(w) & 0xF]) for w in words]


def _stream(stream):
    """hipStream_t handle of a torch stream (or a raw handle); None: NULL."""
    if stream is None:
        return None
    return int(getattr(stream, "cuda_stream", stream)) or None


def swx_align(profile: int, ref, flags: int = SWX_ALL, mask_len: int = -1, stream=None):
    """Align one reference (numpy int8, or a device pointer with its length as a
    tuple (ptr, rlen) and flags | SWX_REF_DEVICE) on `stream` (a torch stream,
    a raw hipStream_t, or None for the context's own).  Returns (record dict,
    cigar list), and with SWX_SUBOPT also the suboptimal alignment's (record
    dict, cigar list)."""
    res = SwxResult()
    if isinstance(ref, tuple):
        ptr, rlen = ref
        st = lib().swx_align(profile, ctypes.c_void_p(ptr), int(rlen), int(flags),
                             int(mask_len), _stream(stream), ctypes.byref(res))
    else:
        r = np.ascontiguousarray(ref, dtype=np.int8)
        st = lib().swx_align(profile, r.ctypes.data if len(r) else None, len(r), int(flags),
                             int(mask_len), _stream(stream), ctypes.byref(res))
    _check(st, "swx_align")
    rec = {k: getattr(res.rec, k) for k, _ in SwxRec._fields_}
    cig = [res.cigar[k] for k in range(res.rec.cigar_len)] if res.rec.cigar_len else []
    sub = {k: getattr(res.sub, k) for k, _ in SwxRec._fields_}
    scig = [res.sub_cigar[k] for k in range(res.sub.cigar_len)] if res.sub.cigar_len else []
    lib().swx_result_free(ctypes.byref(res))
    if flags & SWX_SUBOPT:
        return rec, decode_cigar(cig), sub, decode_cigar(scig)
    return rec, decode_cigar(cig)


def swx_result_free(res) -> None:
    lib().swx_result_free(ctypes.byref(res))


def swx_strerror(status: int) -> str:
    return lib().swx_strerror(int(status)).decode()


def swx_last_error() -> str:
    return lib().swx_last_error().decode(errors="replace")


def swx_last_stage_ms(ctx: int, cap: int = 8) -> list:
    buf = (ctypes.c_double * cap)()
    n = lib().swx_last_stage_ms(ctx, buf, cap)
    if n < 0:
        raise SwxError(n, "swx_last_stage_ms")
    return [buf[k] for k in range(n)]


def swx_get_tuning(ctx: int) -> dict:
    t = SwxTuning()
    _check(lib().swx_get_tuning(ctx, ctypes.byref(t)), "swx_get_tuning")
    return {k: getattr(t, k) for k, _ in SwxTuning._fields_ if k != "pad_"}


def swx_set_tuning(ctx: int, **changes) -> None:
    """Change some knobs of the launch configuration, keeping the others."""
    cur = swx_get_tuning(ctx)
    unknown = set(changes) - set(cur)
    if unknown:
        raise KeyError(f"unknown tuning keys {sorted(unknown)}")
    cur.update(changes)
    t = SwxTuning(**cur)
    _check(lib().swx_set_tuning(ctx, ctypes.byref(t)), "swx_set_tuning")


def _ptr(x):
    """Address of a numpy array or a torch tensor (host or device)."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return x.ctypes.data


def _make_batch(matrix, o, e, qcat, qoff, rcat, roff, pair_q, pair_r, flags, mask_len, in_mem):
    m = np.ascontiguousarray(matrix, dtype=np.int8)
    b = SwxBatch()
    b.matrix = m.ctypes.data
    b.n = int(m.shape[0])
    b.gap_open = int(o)
    b.gap_extend = int(e)
    b.qcat = _ptr(qcat)
    b.qcat_len = int(qcat.numel() if hasattr(qcat, "numel") else len(qcat))
    b.qoff = _ptr(qoff)
    b.nq = int((qoff.numel() if hasattr(qoff, "numel") else len(qoff)) - 1)
    b.rcat = _ptr(rcat)
    b.rcat_len = int(rcat.numel() if hasattr(rcat, "numel") else len(rcat))
    b.roff = _ptr(roff)
    b.nr = int((roff.numel() if hasattr(roff, "numel") else len(roff)) - 1)
    b.pair_q = _ptr(pair_q)
    b.pair_r = _ptr(pair_r)
    b.npairs = int(pair_q.numel() if hasattr(pair_q, "numel") else len(pair_q))
    b.flags = int(flags)
    b.mask_len = int(mask_len)
    b.in_mem = int(in_mem)
    return b, m


def swx_cigar_bound(matrix, o, e, qcat, qoff, rcat, roff, pair_q, pair_r, flags=0) -> int:
    arrs = [np.ascontiguousarray(x, dtype=np.int64) for x in (qoff, roff, pair_q, pair_r)]
    qc = np.ascontiguousarray(qcat, dtype=np.int8)
    rc = np.ascontiguousarray(rcat, dtype=np.int8)
    b, _m = _make_batch(matrix, o, e, qc, arrs[0], rc, arrs[1], arrs[2], arrs[3], flags, -1,
                        SWX_MEM_HOST)
    return int(lib().swx_cigar_bound(ctypes.byref(b)))


def swx_align_batch(ctx: int, matrix, o, e, qcat, qoff, rcat, roff, pair_q, pair_r,
                    flags=SWX_ALL, mask_len=-1, in_mem=SWX_MEM_HOST, recs=None, cigar=None,
                    out_mem=SWX_MEM_HOST, sub_recs=None, stream=None):
    """Raw batch call.  Host-memory inputs are numpy arrays; device-memory
    inputs are torch tensors.  recs/cigar are caller-owned outputs (numpy
    structured array of REC_DTYPE and uint32 array on the host, or torch
    tensors on the device).  stream: a torch stream or raw hipStream_t the
    call's work is queued on (None: the context's own).  Returns (status,
    cigar_used)."""
    return _batch_call(lib().swx_align_batch, ctx, matrix, o, e, qcat, qoff, rcat, roff, pair_q,
                       pair_r, flags, mask_len, in_mem, recs, cigar, out_mem, sub_recs, stream)


def swx_align_batch_noalloc(ctx: int, matrix, o, e, qcat, qoff, rcat, roff, pair_q, pair_r,
                            flags=SWX_ALL, mask_len=-1, in_mem=SWX_MEM_HOST, recs=None,
                            cigar=None, out_mem=SWX_MEM_HOST, stream=None):
    """The batch call that allocates no device memory (its scratch is the
    library's static per-GPU array).  Arguments as swx_align_batch."""
    return _batch_call(lib().swx_align_batch_noalloc, ctx, matrix, o, e, qcat, qoff, rcat, roff,
                       pair_q, pair_r, flags, mask_len, in_mem, recs, cigar, out_mem, None,
                       stream)


def _batch_call(fn, ctx, matrix, o, e, qcat, qoff, rcat, roff, pair_q, pair_r, flags, mask_len,
                in_mem, recs, cigar, out_mem, sub_recs, stream):
    b, _m = _make_batch(matrix, o, e, qcat, qoff, rcat, roff, pair_q, pair_r, flags, mask_len,
                        in_mem)
    out = SwxBatchOut()
    out.recs = _ptr(recs)
    out.cigar = _ptr(cigar)
    out.cigar_cap = int(cigar.numel() if hasattr(cigar, "numel") else
                        (len(cigar) if cigar is not None else 0))
    out.out_mem = int(out_mem)
    out.sub_recs = _ptr(sub_recs)
    st = fn(ctx, ctypes.byref(b), ctypes.byref(out), _stream(stream))
    return st, int(out.cigar_used)


class Context:
    """One library context (device stream + memory pool)."""

    def __init__(self, device: int = 0):
        self.handle = swx_ctx_create(device)

    def close(self):
        if self.handle:
            swx_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def lane_probe(self, bits, columns=4096, blocks=2048, o=3, e=1):
        """swx_lane_probe: (best scores per synthetic pair, kernel ms, GCUPS)."""
        n = blocks * 256 * (32 // bits)
        best = np.zeros(n, dtype=np.uint32)
        ms = ctypes.c_double()
        _check(lib().swx_lane_probe(self.handle, bits, columns, blocks, o, e, best.ctypes.data,
                                    ctypes.byref(ms)), "swx_lane_probe")
        cells = n * 16 * columns
        return best, ms.value, cells / (ms.value * 1e-3) / 1e9

    def check_max3(self):
        """swx_check_max3: (mismatches, results compared)."""
        bad, n = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().swx_check_max3(self.handle, ctypes.byref(bad), ctypes.byref(n)), "swx_check_max3")
        return bad.value, n.value

    def stage_ms(self):
        return swx_last_stage_ms(self.handle)

    def autotune(self, matrix, o, e, qcat, qoff, rcat, roff, pair_q, pair_r, max_pairs=65536,
                 cache_path=None, in_mem=SWX_MEM_HOST):
        """Times the launch configurations on a sample of the batch (numpy
        arrays on the host, or torch tensors on the device with in_mem =
        SWX_MEM_DEVICE) and installs the fastest.  Returns (tuning, from_cache)."""
        if in_mem == SWX_MEM_HOST:
            qcat = np.ascontiguousarray(qcat, dtype=np.int8)
            rcat = np.ascontiguousarray(rcat, dtype=np.int8)
            qoff, roff, pair_q, pair_r = (np.ascontiguousarray(x, dtype=np.int64)
                                          for x in (qoff, roff, pair_q, pair_r))
        b, _m = _make_batch(matrix, o, e, qcat, qoff, rcat, roff, pair_q, pair_r, SWX_ALL, -1,
                            in_mem)
        t = SwxTuning()
        fc = ctypes.c_int32()
        path = cache_path.encode() if cache_path else None
        _check(lib().swx_autotune(self.handle, ctypes.byref(b), int(max_pairs), path,
                                  ctypes.byref(t), ctypes.byref(fc)), "swx_autotune")
        return {k: getattr(t, k) for k, _ in SwxTuning._fields_ if k != "pad_"}, bool(fc.value)

    def tuning(self) -> dict:
        return swx_get_tuning(self.handle)

    def set_tuning(self, **changes) -> None:
        swx_set_tuning(self.handle, **changes)

    def align_pair(self, query, ref, matrix, o, e, flags=SWX_ALL, mask_len=-1, stream=None):
        p = swx_profile_create(self.handle, query, matrix, o, e)
        try:
            return swx_align(p, ref, flags, mask_len, stream)
        finally:
            swx_profile_destroy(p)

    def align_batch(self, matrix, o, e, qcat, qoff, rcat, roff, pair_q, pair_r,
                    flags=SWX_ALL, mask_len=-1):
        """Host-memory batch: returns (records [REC_DTYPE], cigar words), and
        with SWX_SUBOPT (records, cigar words, suboptimal records)."""
        qcat = np.ascontiguousarray(qcat, dtype=np.int8)
        rcat = np.ascontiguousarray(rcat, dtype=np.int8)
        qoff, roff, pair_q, pair_r = (np.ascontiguousarray(x, dtype=np.int64)
                                      for x in (qoff, roff, pair_q, pair_r))
        npairs = len(pair_q)
        recs = np.zeros(npairs, dtype=REC_DTYPE)
        sub = np.zeros(npairs, dtype=REC_DTYPE) if flags & SWX_SUBOPT else None
        cap = swx_cigar_bound(matrix, o, e, qcat, qoff, rcat, roff, pair_q, pair_r, flags)
        cig = np.zeros(max(cap, 1), dtype=np.uint32)
        st, used = swx_align_batch(self.handle, matrix, o, e, qcat, qoff, rcat, roff, pair_q,
                                   pair_r, flags, mask_len, SWX_MEM_HOST, recs, cig, SWX_MEM_HOST,
                                   sub)
        _check(st, "swx_align_batch")
        return (recs, cig[:used]) if sub is None else (recs, cig[:used], sub)


    def align_batch_chunks(self, matrix, o, e, qcat, qoff, rcat, roff, pair_q, pair_r,
                           chunk_pairs, cigar_words_per_pair=16, flags=SWX_ALL, mask_len=-1,
                           stream=None):
        """A pair list of any length in slices: yields (k0, k1, recs, cigar)
        for each slice [k0, k1) of at most chunk_pairs pairs, computed by one
        swx_align_batch call each.  Inputs are either all numpy arrays (host)
        or all torch tensors on the context's device (device-resident; the
        pair lists are sliced as views).  recs (chunk_pairs records) and the
        CIGAR arena are reused from slice to slice -- consume or copy them
        before the next one -- so the device memory held stays at one
        slice's outputs however many pairs there are; a slice whose CIGARs
        outgrow the arena (cigar_words_per_pair words per pair to start with)
        is run again with one that fits.  recs[:k1 - k0] and cigar[:used] are
        the slice's records (cigar_off relative to the slice's arena) and
        CIGAR words."""
        dev = hasattr(pair_q, "data_ptr")
        npairs = int(pair_q.numel() if dev else len(pair_q))
        chunk_pairs = max(1, int(chunk_pairs))
        cap = max(1, min(chunk_pairs, npairs) * int(cigar_words_per_pair))
        if dev:
            import torch
            recs = torch.empty(min(chunk_pairs, npairs) * REC_DTYPE.itemsize, dtype=torch.uint8,
                               device=pair_q.device)
            cig = torch.empty(cap, dtype=torch.int32, device=pair_q.device)
            mem = SWX_MEM_DEVICE
        else:
            qcat = np.ascontiguousarray(qcat, dtype=np.int8)
            rcat = np.ascontiguousarray(rcat, dtype=np.int8)
            qoff, roff, pair_q, pair_r = (np.ascontiguousarray(x, dtype=np.int64)
                                          for x in (qoff, roff, pair_q, pair_r))
            recs = np.zeros(min(chunk_pairs, npairs), dtype=REC_DTYPE)
            cig = np.zeros(cap, dtype=np.uint32)
            mem = SWX_MEM_HOST
        for k0 in range(0, npairs, chunk_pairs):
            k1 = min(npairs, k0 + chunk_pairs)
            pq, pr = pair_q[k0:k1], pair_r[k0:k1]
            while True:
                st, used = swx_align_batch(self.handle, matrix, o, e, qcat, qoff, rcat, roff, pq,
                                           pr, flags, mask_len, mem, recs, cig, mem, None, stream)
                if st == SWX_ERANGE and used > cap:
                    cap = used
                    if dev:
                        import torch
                        cig = torch.empty(cap, dtype=torch.int32, device=pair_q.device)
                    else:
                        cig = np.zeros(cap, dtype=np.uint32)
                    continue
                _check(st, "swx_align_batch")
                break
            yield k0, k1, recs, cig[:used]


# ---- graph mode ---------------------------------------------------------------
class Graph:
    """The batched path captured as one hipGraph for batches of a fixed
    capacity (swx_graph_*): load a host batch, run (replay), read results."""

    def __init__(self, ctx: "Context", matrix, o, e, max_pairs, max_qlen, max_rlen, qcat_cap,
                 rcat_cap, nq_cap, nr_cap, flags=SWX_ALL, mask_len=-1, route=0):
        self._m = np.ascontiguousarray(matrix, dtype=np.int8)
        cfg = SwxGraphCfg(matrix=self._m.ctypes.data, n=self._m.shape[0], gap_open=o,
                          gap_extend=e, max_pairs=max_pairs, max_qlen=max_qlen, pad_=0,
                          max_rlen=max_rlen, qcat_cap=qcat_cap, rcat_cap=rcat_cap, nq_cap=nq_cap,
                          nr_cap=nr_cap, flags=flags, mask_len=mask_len, route=route, pad2_=0)
        h = ctypes.c_void_p()
        self.io = SwxGraphIo()
        _check(lib().swx_graph_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h),
                                      ctypes.byref(self.io)), "swx_graph_create")
        self.handle = h.value
        self.ctx = ctx
        self.max_pairs = max_pairs
        self.npairs = 0

    def load(self, qcat, qoff, rcat, roff, pair_q, pair_r):
        qcat = np.ascontiguousarray(qcat, dtype=np.int8)
        rcat = np.ascontiguousarray(rcat, dtype=np.int8)
        qoff, roff, pair_q, pair_r = (np.ascontiguousarray(x, dtype=np.int64)
                                      for x in (qoff, roff, pair_q, pair_r))
        b, _mm = _make_batch(self._m, 0, 0, qcat, qoff, rcat, roff, pair_q, pair_r, 0, -1,
                             SWX_MEM_HOST)
        _check(lib().swx_graph_load(self.handle, ctypes.byref(b)), "swx_graph_load")
        self.npairs = len(pair_q)

    def run(self, eager=False, stream=None):
        f = lib().swx_graph_run_eager if eager else lib().swx_graph_run
        _check(f(self.handle, _stream(stream)), "swx_graph_run")

    def read(self):
        recs = np.zeros(self.npairs, dtype=REC_DTYPE)
        cig = np.zeros(max(int(self.io.cigar_cap), 1), dtype=np.uint32)
        out = SwxBatchOut()
        out.recs = recs.ctypes.data
        out.cigar = cig.ctypes.data
        out.cigar_cap = len(cig)
        out.out_mem = SWX_MEM_HOST
        _check(lib().swx_graph_read(self.handle, self.npairs, ctypes.byref(out)), "swx_graph_read")
        return recs, cig[:out.cigar_used]

    def close(self):
        if self.handle:
            _check(lib().swx_graph_destroy(self.handle), "swx_graph_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- serving ------------------------------------------------------------------
SWX_EBUSY = -4


class Server:
    """Request loop (swx_server_*): resident queries, footprint admission,
    continuous batching.  Requests are submitted as REQ_DTYPE arrays whose
    pointers refer to host code arrays the caller keeps alive until submit
    returns (the library copies them)."""

    def __init__(self, matrix, o, e, device=0, mem_budget=0, max_pending=0, workers=0,
                 max_batch=0, flags=SWX_ALL, mask_len=-1, long_cells=0, graph_batch=0,
                 graph_max_qlen=0, graph_max_rlen=0, side_streams=-1):
        self._m = np.ascontiguousarray(matrix, dtype=np.int8)
        cfg = SwxServerCfg(device=device, matrix=self._m.ctypes.data, n=self._m.shape[0],
                           gap_open=o, gap_extend=e, mem_budget=mem_budget,
                           max_pending=max_pending, workers=workers, max_batch=max_batch,
                           flags=flags, mask_len=mask_len, long_cells=long_cells,
                           graph_batch=graph_batch, graph_max_qlen=graph_max_qlen,
                           graph_max_rlen=graph_max_rlen, side_streams=side_streams)
        h = ctypes.c_void_p()
        _check(lib().swx_server_create(ctypes.byref(cfg), ctypes.byref(h)), "swx_server_create")
        self.handle = h.value

    def register_query(self, query) -> int:
        q = np.ascontiguousarray(query, dtype=np.int8)
        qid = ctypes.c_int64()
        _check(lib().swx_server_register_query(self.handle, q.ctypes.data, len(q),
                                               ctypes.byref(qid)), "swx_server_register_query")
        return qid.value

    def submit(self, reqs: np.ndarray):
        """Submit a REQ_DTYPE array.  Returns (status, tickets of the accepted prefix)."""
        reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
        tickets = np.zeros(len(reqs), dtype=np.uint64)
        acc = ctypes.c_int32()
        st = lib().swx_server_submit(self.handle, reqs.ctypes.data, len(reqs),
                                     tickets.ctypes.data, ctypes.byref(acc))
        if st not in (SWX_OK, SWX_EBUSY):
            raise SwxError(st, "swx_server_submit")
        return st, tickets[:acc.value]

    def poll(self, max_n=4096, timeout_us=0, keep_cigar=False):
        """Finished completions as a COMPLETION_DTYPE array (and, with
        keep_cigar, a list of CIGAR word arrays).  CIGAR memory is released."""
        buf = np.zeros(max_n, dtype=COMPLETION_DTYPE)
        nd = ctypes.c_int32()
        _check(lib().swx_server_poll(self.handle, buf.ctypes.data, max_n, int(timeout_us),
                                     ctypes.byref(nd)), "swx_server_poll")
        out = buf[:nd.value].copy()
        cigs = None
        if keep_cigar:
            cigs = []
            for c in out:
                n = int(c["rec"]["cigar_len"])
                if n and c["cigar"]:
                    arr = (ctypes.c_uint32 * n).from_address(int(c["cigar"]))
                    cigs.append(np.frombuffer(arr, dtype=np.uint32).copy())
                else:
                    cigs.append(np.zeros(0, dtype=np.uint32))
        lib().swx_completion_free(buf.ctypes.data, nd.value)
        return (out, cigs) if keep_cigar else out

    def stats(self) -> dict:
        t = SwxServerStats()
        _check(lib().swx_server_stats_get(self.handle, ctypes.byref(t)), "swx_server_stats_get")
        return {k: getattr(t, k) for k, _ in SwxServerStats._fields_}

    def close(self):
        if self.handle:
            _check(lib().swx_server_destroy(self.handle), "swx_server_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SIM_REQ_DTYPE = np.dtype([("arrival_us", "<f8"), ("qlen", "<i8"), ("rlen", "<i8")])
SIM_RESULT_DTYPE = np.dtype([("start_us", "<f8"), ("done_us", "<f8"), ("batch_id", "<i8"),
                             ("footprint", "<i8"), ("worker", "<i4"), ("batch_size", "<i4"),
                             ("cls", "<i4"), ("status", "<i4")])


def simulate_serving(arrival_us, qlen, rlen, cells_per_us, batch_us=0.0, request_us=0.0, n=4,
                     mem_budget=0, max_pending=0, workers=0, max_batch=0, long_cells=0):
    """swx_server_simulate: the serving policy on a virtual clock against a
    modelled GPU (no device needed).  Returns (SIM_RESULT_DTYPE array, stats)."""
    rq = np.zeros(len(arrival_us), dtype=SIM_REQ_DTYPE)
    rq["arrival_us"] = arrival_us
    rq["qlen"] = qlen
    rq["rlen"] = rlen
    out = np.zeros(len(rq), dtype=SIM_RESULT_DTYPE)
    cfg = SwxServerCfg(device=0, matrix=None, n=n, gap_open=1, gap_extend=1,
                       mem_budget=mem_budget, max_pending=max_pending, workers=workers,
                       max_batch=max_batch, flags=0, mask_len=-1, long_cells=long_cells)
    model = SwxSimModel(cells_per_us=cells_per_us, batch_us=batch_us, request_us=request_us)
    st = SwxServerStats()
    _check(lib().swx_server_simulate(ctypes.byref(cfg), ctypes.byref(model), rq.ctypes.data,
                                     len(rq), out.ctypes.data, ctypes.byref(st)),
           "swx_server_simulate")
    return out, {k: getattr(st, k) for k, _ in SwxServerStats._fields_}


def make_requests(qcat, qoff, rcat, roff, pair_q, pair_r, tags=None, query_ids=None):
    """REQ_DTYPE array for pairs over concatenated host arrays (which must stay
    alive until submit returns)."""
    qcat = np.ascontiguousarray(qcat, dtype=np.int8)
    rcat = np.ascontiguousarray(rcat, dtype=np.int8)
    pair_q = np.asarray(pair_q, dtype=np.int64)
    pair_r = np.asarray(pair_r, dtype=np.int64)
    qoff = np.asarray(qoff, dtype=np.int64)
    roff = np.asarray(roff, dtype=np.int64)
    r = np.zeros(len(pair_q), dtype=REQ_DTYPE)
    r["query_id"] = -1 if query_ids is None else query_ids
    r["query"] = qcat.ctypes.data + qoff[pair_q]
    r["qlen"] = qoff[pair_q + 1] - qoff[pair_q]
    r["ref"] = rcat.ctypes.data + roff[pair_r]
    r["rlen"] = roff[pair_r + 1] - roff[pair_r]
    r["tag"] = np.arange(len(pair_q)) if tags is None else tags
    return r
