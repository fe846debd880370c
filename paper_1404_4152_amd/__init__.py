"""Python binding of libswmi (exact Smith-Waterman database search on gfx950).

Argument marshalling only: every step of the search runs in the HIP kernels
of ``libswmi.so``; this module converts numpy arrays to pointers and return
codes to exceptions.  Function names match the C ABI in ``include/swmi.h``.
There is no CPU fallback: if the library is missing, importing the binding's
functions raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SWMI_LIB") or os.path.join(HERE, "libswmi.so")

SW_OK, SW_EINVAL, SW_ENOMEM, SW_EDEVICE, SW_EBUSY, SW_ENOTFOUND, SW_ESTOPPED = 0, -1, -2, -3, -4, -5, -6
SW_TIER_AUTO, SW_TIER_F16X2, SW_TIER_I16X2 = 0, 1, 2
SW_PROFILE_PAIR, SW_PROFILE_SCORE = 0, 1
SW_MAX_K = 4096
SW_MAX_ALPHABET = 32


class SwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class sw_scoring(ctypes.Structure):
    _fields_ = [("alphabet", ctypes.c_int32), ("matrix", ctypes.POINTER(ctypes.c_int8)),
                ("alpha", ctypes.c_int32), ("beta", ctypes.c_int32)]


class sw_db_opts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("long_threshold", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 6)]


class sw_search_opts(ctypes.Structure):
    _fields_ = [("tier", ctypes.c_int32), ("strip", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("sat_threshold", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class sw_stats(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_int64), ("padded_cells", ctypes.c_int64),
                ("inter_cells", ctypes.c_int64), ("recomputed_pairs", ctypes.c_int64), ("intra_pairs", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("inter_ms", ctypes.c_double), ("tier", ctypes.c_int32), ("strip", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("graphed", ctypes.c_int32),
                ("fused_long", ctypes.c_int32), ("recompute_ms", ctypes.c_double),
                ("long_ms", ctypes.c_double), ("profile", ctypes.c_int32),
                ("reserved0", ctypes.c_int32)]


class sw_alignment(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int32), ("q_begin", ctypes.c_int32), ("q_end", ctypes.c_int32),
                ("n_ops", ctypes.c_int32), ("s_begin", ctypes.c_int64), ("s_end", ctypes.c_int64),
                ("ops_offset", ctypes.c_int64)]


class sw_server_opts(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_int64), ("max_active", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("chunk_groups", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 5)]


class sw_req_stats(ctypes.Structure):
    _fields_ = [("queue_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("cells", ctypes.c_int64), ("passes", ctypes.c_int32),
                ("shared_passes", ctypes.c_int32)]


class sw_index_opts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("memory_budget", ctypes.c_int64), ("reserved", ctypes.c_int32 * 4)]


class sw_index_stats(ctypes.Structure):
    _fields_ = [("chunks", ctypes.c_int64), ("resident", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("bytes_loaded", ctypes.c_int64),
                ("cells", ctypes.c_int64), ("load_ms", ctypes.c_double),
                ("search_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double)]


_P = ctypes.POINTER
_u8p, _i8p, _i32p, _i64p = _P(ctypes.c_uint8), _P(ctypes.c_int8), _P(ctypes.c_int32), _P(ctypes.c_int64)
_vp = ctypes.c_void_p

# name -> (restype, argtypes), in the order of include/swmi.h
SIGNATURES = {
    "sw_db_open": (ctypes.c_int, [_u8p, _i64p, ctypes.c_int64, ctypes.c_int32, _P(sw_db_opts), _P(_vp)]),
    "sw_db_close": (None, [_vp]),
    "sw_db_size": (ctypes.c_int64, [_vp]),
    "sw_db_set_opts": (ctypes.c_int, [_vp, _P(sw_search_opts)]),
    "sw_db_last_stats": (ctypes.c_int, [_vp, _P(sw_stats)]),
    "sw_db_search": (ctypes.c_int, [_vp, _u8p, ctypes.c_int32, _P(sw_scoring), _i32p, _vp]),
    "sw_db_search_dev": (ctypes.c_int, [_vp, _u8p, ctypes.c_int32, _P(sw_scoring), _vp, _vp]),
    "sw_db_search_dev_noalloc": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, _P(sw_scoring), _vp, _vp]),
    "sw_db_topk": (ctypes.c_int, [_vp, _u8p, ctypes.c_int32, _P(sw_scoring), ctypes.c_int32, _i32p,
                                  _i64p, _vp]),
    "sw_db_search_batch": (ctypes.c_int, [_vp, ctypes.c_int32, _u8p, _i64p, _P(sw_scoring),
                                          ctypes.c_int32, _i32p, _i64p, _i32p, _vp]),
    "sw_db_autotune": (ctypes.c_int, [_vp, _P(sw_scoring), _i32p, ctypes.c_int32, ctypes.c_char_p]),
    "sw_db_align": (ctypes.c_int, [_vp, _u8p, ctypes.c_int32, _P(sw_scoring), _i64p, ctypes.c_int32,
                                   _P(sw_alignment), _P(ctypes.c_uint32), ctypes.c_int64, _i64p]),
    "sw_server_start": (ctypes.c_int, [_vp, _P(sw_server_opts), _P(_vp)]),
    "sw_server_submit": (ctypes.c_int, [_vp, _u8p, ctypes.c_int32, _P(sw_scoring), ctypes.c_int32,
                                        _P(ctypes.c_uint64)]),
    "sw_server_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, _i32p, _i64p, _P(sw_req_stats)]),
    "sw_server_stop": (None, [_vp]),
    "sw_index_write": (ctypes.c_int, [ctypes.c_char_p, _u8p, _i64p, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_int64]),
    "sw_index_open": (ctypes.c_int, [ctypes.c_char_p, _P(sw_index_opts), _P(_vp)]),
    "sw_index_close": (None, [_vp]),
    "sw_index_size": (ctypes.c_int64, [_vp]),
    "sw_index_last_stats": (ctypes.c_int, [_vp, _P(sw_index_stats)]),
    "sw_index_search_batch": (ctypes.c_int, [_vp, ctypes.c_int32, _u8p, _i64p, _P(sw_scoring),
                                             ctypes.c_int32, _i32p, _i64p, _i32p]),
    "sw_last_error": (ctypes.c_char_p, []),
    "sw_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """The loaded libswmi.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7, and
        # the library's streams and device pointers must live in the same
        # runtime as the caller's tensors and streams.  Loading torch first makes
        # libswmi bind to that runtime instead of a second copy from /opt/rocm.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python paper_1404_4152_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != SW_OK:
        raise SwError(rc, lib().sw_last_error().decode())
    return rc


def _ptr(a, ctype):
    return a.ctypes.data_as(_P(ctype))


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a if a.size else np.zeros(1, np.uint8)


def make_scoring(matrix, alpha, beta):
    """(sw_scoring, keepalive) for an int8 matrix whose row is the query residue."""
    m = np.ascontiguousarray(matrix, dtype=np.int8)
    sc = sw_scoring(m.shape[0], _ptr(m, ctypes.c_int8), int(alpha), int(beta))
    return sc, m


# ---------------------------------------------------------------------------
# C-named wrappers
# ---------------------------------------------------------------------------
def sw_version() -> str:
    return lib().sw_version().decode()


def sw_last_error() -> str:
    return lib().sw_last_error().decode()


def sw_db_open(residues, offsets, alphabet, long_threshold=0, device=0):
    res = _u8(residues)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    opts = sw_db_opts(device, long_threshold)
    h = _vp()
    _check(lib().sw_db_open(_ptr(res, ctypes.c_uint8), _ptr(off, ctypes.c_int64), len(off) - 1,
                            int(alphabet), ctypes.byref(opts), ctypes.byref(h)))
    return h


def sw_db_close(h):
    lib().sw_db_close(h)


def sw_db_size(h) -> int:
    return int(lib().sw_db_size(h))


def sw_db_set_opts(h, tier=0, strip=0, waves=0, sat_threshold=0, graph=0, profile=0, reset=False):
    if reset:
        return _check(lib().sw_db_set_opts(h, None))
    o = sw_search_opts(tier, strip, waves, sat_threshold, graph, profile)
    return _check(lib().sw_db_set_opts(h, ctypes.byref(o)))


def sw_db_last_stats(h) -> dict:
    s = sw_stats()
    _check(lib().sw_db_last_stats(h, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in sw_stats._fields_ if not f.startswith("reserved")}


def sw_db_search(h, query, matrix, alpha, beta, stream=None):
    n = sw_db_size(h)
    out = np.zeros(max(n, 1), dtype=np.int32)
    q = _u8(query)
    sc, keep = make_scoring(matrix, alpha, beta)
    _check(lib().sw_db_search(h, _ptr(q, ctypes.c_uint8), len(query), ctypes.byref(sc),
                              _ptr(out, ctypes.c_int32), stream))
    return out[:n]


def sw_db_search_dev(h, query, matrix, alpha, beta, scores_dev_ptr: int, stream=None):
    q = _u8(query)
    sc, keep = make_scoring(matrix, alpha, beta)
    return _check(lib().sw_db_search_dev(h, _ptr(q, ctypes.c_uint8), len(query), ctypes.byref(sc),
                                         ctypes.c_void_p(scores_dev_ptr), stream))


def sw_db_search_dev_noalloc(h, query_dev_ptr: int, qlen: int, matrix, alpha, beta,
                             scores_dev_ptr: int, stream=None):
    sc, keep = make_scoring(matrix, alpha, beta)
    return _check(lib().sw_db_search_dev_noalloc(h, ctypes.c_void_p(query_dev_ptr), int(qlen),
                                                 ctypes.byref(sc), ctypes.c_void_p(scores_dev_ptr),
                                                 stream))


def sw_db_topk(h, query, matrix, alpha, beta, k, stream=None):
    q = _u8(query)
    sc, keep = make_scoring(matrix, alpha, beta)
    ts = np.zeros(k, np.int32)
    ti = np.zeros(k, np.int64)
    _check(lib().sw_db_topk(h, _ptr(q, ctypes.c_uint8), len(query), ctypes.byref(sc), int(k),
                            _ptr(ts, ctypes.c_int32), _ptr(ti, ctypes.c_int64), stream))
    return ts, ti


def pack_queries(queries):
    lens = np.array([len(q) for q in queries], np.int64)
    off = np.zeros(len(queries) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    res = np.concatenate([np.asarray(q, np.uint8) for q in queries]) if queries else np.zeros(0, np.uint8)
    return res, off


def sw_db_search_batch(h, queries, matrix, alpha, beta, k, all_scores=False, stream=None):
    res, off = pack_queries(queries)
    res = _u8(res)
    nq = len(queries)
    sc, keep = make_scoring(matrix, alpha, beta)
    ts = np.zeros(nq * k, np.int32)
    ti = np.zeros(nq * k, np.int64)
    n = sw_db_size(h)
    al = np.zeros(max(nq * n, 1), np.int32) if all_scores else None
    _check(lib().sw_db_search_batch(h, nq, _ptr(res, ctypes.c_uint8), _ptr(off, ctypes.c_int64),
                                    ctypes.byref(sc), int(k), _ptr(ts, ctypes.c_int32),
                                    _ptr(ti, ctypes.c_int64),
                                    _ptr(al, ctypes.c_int32) if al is not None else None, stream))
    out = (ts.reshape(nq, k), ti.reshape(nq, k))
    if all_scores:
        out = out + (al[:nq * n].reshape(nq, n),)
    return out


def sw_db_autotune(h, matrix, alpha, beta, qlens, cache_path=None):
    sc, keep = make_scoring(matrix, alpha, beta)
    ql = np.ascontiguousarray(qlens, dtype=np.int32)
    return _check(lib().sw_db_autotune(h, ctypes.byref(sc), _ptr(ql, ctypes.c_int32), len(ql),
                                       cache_path.encode() if cache_path else None))


def sw_db_align(h, query, matrix, alpha, beta, ids):
    """Optimal local alignments of ``query`` against the database sequences
    ``ids``: a list of dicts with score, q_begin, q_end, s_begin, s_end and
    ops, a list of (op, length) runs (op 0 aligned pair, 1 query residue
    against a gap, 2 subject residue against a gap)."""
    q = _u8(query)
    sc, keep = make_scoring(matrix, alpha, beta)
    idv = np.ascontiguousarray(ids, dtype=np.int64)
    n = len(idv)
    out = (sw_alignment * max(n, 1))()
    need = ctypes.c_int64(0)
    if n:
        # a call with no room for runs reports the bound they may need
        rc = lib().sw_db_align(h, _ptr(q, ctypes.c_uint8), len(q), ctypes.byref(sc),
                               _ptr(idv, ctypes.c_int64), n, out, None, 0, ctypes.byref(need))
        if rc != SW_EINVAL or need.value <= 0:
            _check(rc)
    ops = np.zeros(max(need.value, 1), np.uint32)
    _check(lib().sw_db_align(h, _ptr(q, ctypes.c_uint8), len(q), ctypes.byref(sc),
                             _ptr(idv, ctypes.c_int64), n, out, _ptr(ops, ctypes.c_uint32),
                             need.value, ctypes.byref(need)))
    res = []
    for k in range(n):
        o = out[k]
        runs = ops[o.ops_offset:o.ops_offset + o.n_ops]
        res.append({"score": int(o.score), "q_begin": int(o.q_begin), "q_end": int(o.q_end),
                    "s_begin": int(o.s_begin), "s_end": int(o.s_end),
                    "ops": [(int(x & 3), int(x >> 2)) for x in runs]})
    return res


def sw_server_start(h, memory_budget=0, max_active=0, queue_capacity=0, chunk_groups=0):
    o = sw_server_opts(memory_budget, max_active, queue_capacity, chunk_groups)
    s = _vp()
    _check(lib().sw_server_start(h, ctypes.byref(o), ctypes.byref(s)))
    return s


def sw_server_submit(srv, query, matrix, alpha, beta, k):
    q = _u8(query)
    sc, keep = make_scoring(matrix, alpha, beta)
    t = ctypes.c_uint64()
    _check(lib().sw_server_submit(srv, _ptr(q, ctypes.c_uint8), len(query), ctypes.byref(sc),
                                  int(k), ctypes.byref(t)))
    return int(t.value)


def sw_server_wait(srv, ticket, k):
    ts = np.zeros(k, np.int32)
    ti = np.zeros(k, np.int64)
    st = sw_req_stats()
    _check(lib().sw_server_wait(srv, ctypes.c_uint64(ticket), _ptr(ts, ctypes.c_int32),
                                _ptr(ti, ctypes.c_int64), ctypes.byref(st)))
    return ts, ti, {f: getattr(st, f) for f, _ in sw_req_stats._fields_ if f != "reserved"}


def sw_server_stop(srv):
    lib().sw_server_stop(srv)


def sw_index_write(path, residues, offsets, alphabet, chunk_residues):
    res = _u8(residues)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    return _check(lib().sw_index_write(os.fsencode(path), _ptr(res, ctypes.c_uint8),
                                       _ptr(off, ctypes.c_int64), len(off) - 1, int(alphabet),
                                       int(chunk_residues)))


def sw_index_open(path, device=0, memory_budget=0):
    o = sw_index_opts(device, 0, int(memory_budget))
    h = _vp()
    _check(lib().sw_index_open(os.fsencode(path), ctypes.byref(o), ctypes.byref(h)))
    return h


def sw_index_close(h):
    lib().sw_index_close(h)


def sw_index_size(h) -> int:
    return int(lib().sw_index_size(h))


def sw_index_last_stats(h) -> dict:
    st = sw_index_stats()
    _check(lib().sw_index_last_stats(h, ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in sw_index_stats._fields_ if not f.startswith("reserved")}


def sw_index_search_batch(h, queries, matrix, alpha, beta, k, all_scores=False):
    res, off = pack_queries(queries)
    res = _u8(res)
    nq = len(queries)
    sc, keep = make_scoring(matrix, alpha, beta)
    ts = np.zeros(nq * k, np.int32)
    ti = np.zeros(nq * k, np.int64)
    n = sw_index_size(h)
    al = np.zeros(max(nq * n, 1), np.int32) if all_scores else None
    _check(lib().sw_index_search_batch(h, nq, _ptr(res, ctypes.c_uint8), _ptr(off, ctypes.c_int64),
                                       ctypes.byref(sc), int(k), _ptr(ts, ctypes.c_int32),
                                       _ptr(ti, ctypes.c_int64),
                                       _ptr(al, ctypes.c_int32) if al is not None else None))
    out = (ts.reshape(nq, k), ti.reshape(nq, k))
    if all_scores:
        out = out + (al[:nq * n].reshape(nq, n),)
    return out


class Index:
    """An on-disk index searched resident or streamed (closed on ``close``/GC)."""

    def __init__(self, path, device=0, memory_budget=0):
        self.h = sw_index_open(path, device, memory_budget)
        self.n = sw_index_size(self.h)

    def close(self):
        if self.h:
            sw_index_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def search_batch(self, queries, matrix, alpha, beta, k, all_scores=False):
        return sw_index_search_batch(self.h, queries, matrix, alpha, beta, k, all_scores)

    def stats(self):
        return sw_index_last_stats(self.h)


class Database:
    """A database handle with the C calls as methods (closed on ``close``/GC)."""

    def __init__(self, residues, offsets, alphabet, long_threshold=0, device=0):
        self.h = sw_db_open(residues, offsets, alphabet, long_threshold, device)
        self.n = sw_db_size(self.h)

    def close(self):
        if self.h:
            sw_db_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def search(self, query, matrix, alpha, beta):
        return sw_db_search(self.h, query, matrix, alpha, beta)

    def topk(self, query, matrix, alpha, beta, k):
        return sw_db_topk(self.h, query, matrix, alpha, beta, k)

    def search_batch(self, queries, matrix, alpha, beta, k, all_scores=False):
        return sw_db_search_batch(self.h, queries, matrix, alpha, beta, k, all_scores)

    def align(self, query, matrix, alpha, beta, ids):
        return sw_db_align(self.h, query, matrix, alpha, beta, ids)

    def set_opts(self, **kw):
        return sw_db_set_opts(self.h, **kw)

    def stats(self):
        return sw_db_last_stats(self.h)
