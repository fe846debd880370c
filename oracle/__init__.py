"""CPU oracle for Smith-Waterman database search — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never does, and the two
share no code: the oracle is the scalar C in ``sw_oracle.c`` (Eq. 1 of
section II.A followed literally, int32) plus the top-k ordering below.

Top-k (stage iv of the workflow in section III sorts all scores in
descending order; the order among equal scores is not given there): equal
scores are ordered by ascending database index, i.e. a stable sort of
``-score``.  ``k`` larger than the database yields the whole database followed
by ``(-1, -1)`` fill entries.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "sw_oracle.c")
LIB = os.path.join(_HERE, "libsw_oracle.so")

CFLAGS = ["-O2", "-fno-tree-vectorize", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle with gcc (plain scalar C, OpenMP over subjects)."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, src], check=True)
    os.replace(tmp, out)
    return out


class Oracle:
    """ctypes view of one compiled oracle library."""

    def __init__(self, path: str = LIB):
        lib = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i8p = ctypes.POINTER(ctypes.c_int8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.oracle_sw_score.restype = i32
        lib.oracle_sw_score.argtypes = [u8p, i32, u8p, i64, i8p, i32, i32, i32]
        lib.oracle_search.restype = None
        lib.oracle_search.argtypes = [u8p, i32, u8p, i64p, i64, i8p, i32, i32, i32, i32p, i32]
        lib.oracle_search_subset.restype = None
        lib.oracle_search_subset.argtypes = [u8p, i32, u8p, i64p, i64p, i64, i8p, i32, i32,
                                             i32, i32p, i32]
        lib.oracle_sw_align.restype = i64
        lib.oracle_sw_align.argtypes = [u8p, i32, u8p, i64, i8p, i32, i32, i32, i32p, i64p,
                                        ctypes.POINTER(ctypes.c_uint32), i64]
        lib.oracle_max_threads.restype = i32
        lib.oracle_max_threads.argtypes = []
        self._lib = lib
        self.path = path

    @staticmethod
    def _p(a, ctype):
        return a.ctypes.data_as(ctypes.POINTER(ctype))

    def max_threads(self) -> int:
        return int(self._lib.oracle_max_threads())

    def sw_score(self, q, s, matrix, alpha: int, beta: int) -> int:
        """Score of query ``q`` against subject ``s`` (matrix row = query residue)."""
        q = np.ascontiguousarray(q, dtype=np.uint8)
        s = np.ascontiguousarray(s, dtype=np.uint8)
        mat = np.ascontiguousarray(matrix, dtype=np.int8)
        a = mat.shape[0]
        if len(q) == 0:
            q = np.zeros(1, np.uint8)[:0]
        return int(self._lib.oracle_sw_score(
            self._p(q, ctypes.c_uint8), len(q), self._p(s, ctypes.c_uint8), len(s),
            self._p(mat, ctypes.c_int8), a, int(alpha), int(beta)))

    def sw_align(self, q, s, matrix, alpha: int, beta: int) -> dict:
        """Optimal local alignment of ``q`` against ``s`` with traceback (see
        ``oracle_sw_align`` for the tie rules).  Returns score, q_begin, q_end,
        s_begin, s_end (0-based, inclusive; -1 when the score is 0) and ops, a
        list of (op, length) runs: op 0 aligned pair, 1 query residue against a
        gap, 2 subject residue against a gap."""
        q = np.ascontiguousarray(q, dtype=np.uint8)
        s = np.ascontiguousarray(s, dtype=np.uint8)
        mat = np.ascontiguousarray(matrix, dtype=np.int8)
        res = np.zeros(3, np.int32)
        sres = np.zeros(2, np.int64)
        cap = len(q) + len(s) + 1
        ops = np.zeros(cap, np.uint32)
        qq = q if len(q) else np.zeros(1, np.uint8)
        ss = s if len(s) else np.zeros(1, np.uint8)
        n_ops = int(self._lib.oracle_sw_align(
            self._p(qq, ctypes.c_uint8), len(q), self._p(ss, ctypes.c_uint8), len(s),
            self._p(mat, ctypes.c_int8), mat.shape[0], int(alpha), int(beta),
            self._p(res, ctypes.c_int32), self._p(sres, ctypes.c_int64),
            self._p(ops, ctypes.c_uint32), cap))
        if n_ops < 0:
            raise MemoryError("oracle_sw_align failed (%d)" % n_ops)
        return {"score": int(res[0]), "q_begin": int(res[1]), "q_end": int(res[2]),
                "s_begin": int(sres[0]), "s_end": int(sres[1]),
                "ops": [(int(o & 3), int(o >> 2)) for o in ops[:n_ops]]}

    def search(self, q, residues, offsets, matrix, alpha: int, beta: int,
               nthreads: int = 0) -> np.ndarray:
        """Scores of ``q`` against every database sequence, in database order."""
        q = np.ascontiguousarray(q, dtype=np.uint8)
        res = np.ascontiguousarray(residues, dtype=np.uint8)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        mat = np.ascontiguousarray(matrix, dtype=np.int8)
        n = len(off) - 1
        out = np.zeros(n, dtype=np.int32)
        if n == 0:
            return out
        if len(res) == 0:
            res = np.zeros(1, np.uint8)
        self._lib.oracle_search(self._p(q, ctypes.c_uint8), len(q), self._p(res, ctypes.c_uint8),
                                self._p(off, ctypes.c_int64), n, self._p(mat, ctypes.c_int8),
                                mat.shape[0], int(alpha), int(beta),
                                self._p(out, ctypes.c_int32), int(nthreads))
        return out

    def search_subset(self, q, residues, offsets, which, matrix, alpha: int, beta: int,
                      nthreads: int = 0) -> np.ndarray:
        """Scores of ``q`` against the database sequences listed in ``which``."""
        q = np.ascontiguousarray(q, dtype=np.uint8)
        res = np.ascontiguousarray(residues, dtype=np.uint8)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        w = np.ascontiguousarray(which, dtype=np.int64)
        mat = np.ascontiguousarray(matrix, dtype=np.int8)
        out = np.zeros(len(w), dtype=np.int32)
        if len(w) == 0:
            return out
        if len(res) == 0:
            res = np.zeros(1, np.uint8)
        self._lib.oracle_search_subset(self._p(q, ctypes.c_uint8), len(q),
                                       self._p(res, ctypes.c_uint8), self._p(off, ctypes.c_int64),
                                       self._p(w, ctypes.c_int64), len(w),
                                       self._p(mat, ctypes.c_int8), mat.shape[0], int(alpha),
                                       int(beta), self._p(out, ctypes.c_int32), int(nthreads))
        return out


def topk(scores, k: int):
    """Top-k of a score vector: score descending, then index ascending.

    Returns (scores int32[k], indices int64[k]); entries past the end of the
    database are (-1, -1).
    """
    scores = np.asarray(scores, dtype=np.int64)
    order = np.argsort(-scores, kind="stable")[:k]
    top_s = np.full(k, -1, dtype=np.int32)
    top_i = np.full(k, -1, dtype=np.int64)
    top_s[:len(order)] = scores[order]
    top_i[:len(order)] = order
    return top_s, top_i


_default = None


def load(path: str | None = None, rebuild: bool = False) -> Oracle:
    """The compiled oracle (built on first use if the library is missing)."""
    global _default
    if path is not None:
        return Oracle(path)
    if _default is None or rebuild:
        if rebuild or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _default = Oracle(LIB)
    return _default
