"""ctypes loader and build step for the C oracle (oracle/paris_oracle.c). Test infrastructure only."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .breakpoints import breakpoints

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "paris_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, no floating-point contraction)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-fPIC", "-shared", "-o", tmp, SRC, "-lpthread", "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.orc_summarise.argtypes = [P, i64, i32, i32, P, P, P]
        L.orc_ed2.argtypes = [P, P, i64, i32, P]
        L.orc_ed2_at.argtypes = [P, P, i32, P, i64, P]
        L.orc_nn_many.argtypes = [P, i64, P, i64, i32, i32, P, P]
        L.orc_nn_many.restype = ctypes.c_int
        L.orc_lb2.argtypes = [P, P, i64, i32, i32, P, P]
        L.orc_nn_many_blocked.argtypes = [P, i64, P, i64, i32, i32, P, P]
        L.orc_nn_many_blocked.restype = ctypes.c_int
        L.orc_exact_search.argtypes = [P, P, i64, i32, P, i32, P, i64, P, P, P, P, P]
        L.orc_exact_search.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def summarise(X: np.ndarray, w: int = 16):
    X = np.ascontiguousarray(X, dtype=np.float32)
    N, n = X.shape
    beta = np.ascontiguousarray(breakpoints())
    paa = np.empty((N, w), np.float64)
    sym = np.empty((N, w), np.uint8)
    lib().orc_summarise(_p(X), N, n, w, _p(beta), _p(paa), _p(sym))
    return paa, sym


def ed2(q: np.ndarray, X: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.float32)
    out = np.empty(X.shape[0], np.float64)
    lib().orc_ed2(_p(q), _p(X), X.shape[0], X.shape[1], _p(out))
    return out


def ed2_at(q: np.ndarray, X: np.ndarray, idx) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float32)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    if not (X.dtype == np.float32 and X.flags.c_contiguous):
        raise ValueError("X must be C-contiguous float32")
    out = np.empty(idx.shape[0], np.float64)
    lib().orc_ed2_at(_p(q), _p(X), X.shape[1], _p(idx), idx.shape[0], _p(out))
    return out


def nn_many(Q: np.ndarray, X: np.ndarray, threads: int = 1):
    """Brute-force 1-NN of every query; returns (idx int64[M], d2 float64[M], threads used)."""
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    if not (X.dtype == np.float32 and X.flags.c_contiguous):
        raise ValueError("X must be C-contiguous float32")
    M = Q.shape[0]
    idx = np.empty(M, np.int64)
    d2 = np.empty(M, np.float64)
    used = lib().orc_nn_many(_p(Q), M, _p(X), X.shape[0], X.shape[1], threads, _p(idx), _p(d2))
    return idx, d2, max(1, used)


def nn_many_blocked(Q: np.ndarray, X: np.ndarray, threads: int = 1):
    """As ``nn_many`` (bit-identical results), eight queries per pass over the collection."""
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    if not (X.dtype == np.float32 and X.flags.c_contiguous):
        raise ValueError("X must be C-contiguous float32")
    M = Q.shape[0]
    idx = np.empty(M, np.int64)
    d2 = np.empty(M, np.float64)
    used = lib().orc_nn_many_blocked(_p(Q), M, _p(X), X.shape[0], X.shape[1], threads, _p(idx), _p(d2))
    return idx, d2, max(1, used)


class SearchIndex:
    """What the serial exact-search twin needs besides the raw series: the iSAX words and the
    leaf order the approximate search walks (computed by the numpy oracle, once)."""

    def __init__(self, X: np.ndarray, sym: np.ndarray | None = None, mode: str = "root16",
                 seed_cap: int = 16384, n_leaves: int = 4096):
        from .reference import root_offsets, sorted_order
        if not (X.dtype == np.float32 and X.flags.c_contiguous):
            raise ValueError("X must be C-contiguous float32")
        self.X = X
        if sym is None:   # the numpy oracle's words, row blocks on a thread pool
            from concurrent.futures import ThreadPoolExecutor
            from .reference import isax, paa
            sym = np.empty((X.shape[0], 16), np.uint8)

            def block(a):
                sym[a:a + 65536] = isax(paa(X[a:a + 65536]))
            with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
                list(ex.map(block, range(0, X.shape[0], 65536)))
        self.sym = np.ascontiguousarray(sym, dtype=np.uint8)
        self.perm, self.keys = sorted_order(self.sym)
        self.off = root_offsets(self.keys) if mode == "root16" else None
        self.mode, self.seed_cap, self.n_leaves = mode, seed_cap, n_leaves

    def members(self, q: np.ndarray) -> np.ndarray:
        from .reference import query_summary, seed_window
        qs = query_summary(np.asarray(q, np.float32))
        a, b = seed_window(qs, self.keys, self.X.shape[1] // 16, self.mode, self.seed_cap,
                           self.n_leaves, off=self.off)
        return np.ascontiguousarray(self.perm[a:b], dtype=np.int64), qs.paa


def exact_search(q: np.ndarray, ix: "SearchIndex", members=None):
    """Serial exact-search twin in C (one thread); returns (index, squared distance, counters)
    with counters seed_index, lb_survivors, refined, abandoned, bsf_updates. ``members`` (the
    approximate search's leaf and the query PAA) may be passed precomputed."""
    q = np.ascontiguousarray(q, dtype=np.float32)
    mem, qpaa = ix.members(q) if members is None else members
    qpaa = np.ascontiguousarray(qpaa, dtype=np.float64)
    beta = np.ascontiguousarray(breakpoints())
    oi = ctypes.c_int64(-1)
    od = ctypes.c_double(0.0)
    cnt = np.zeros(5, np.int64)
    N, n = ix.X.shape
    rc = lib().orc_exact_search(_p(q), _p(ix.X), N, n, _p(ix.sym), 16, _p(mem), mem.shape[0], _p(qpaa),
                                _p(beta), ctypes.byref(oi), ctypes.byref(od), _p(cnt))
    if rc != 0:
        raise MemoryError("orc_exact_search")
    keys = ("seed_index", "lb_survivors", "refined", "abandoned", "bsf_updates")
    return int(oi.value), float(od.value), dict(zip(keys, (int(v) for v in cnt)))


def lb2(qpaa: np.ndarray, sym: np.ndarray, L: int) -> np.ndarray:
    qpaa = np.ascontiguousarray(qpaa, dtype=np.float64)
    sym = np.ascontiguousarray(sym, dtype=np.uint8)
    beta = np.ascontiguousarray(breakpoints())
    out = np.empty(sym.shape[0], np.float64)
    lib().orc_lb2(_p(qpaa), _p(sym), sym.shape[0], sym.shape[1], L, _p(beta), _p(out))
    return out
