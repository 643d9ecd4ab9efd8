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
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
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


def lb2(qpaa: np.ndarray, sym: np.ndarray, L: int) -> np.ndarray:
    qpaa = np.ascontiguousarray(qpaa, dtype=np.float64)
    sym = np.ascontiguousarray(sym, dtype=np.uint8)
    beta = np.ascontiguousarray(breakpoints())
    out = np.empty(sym.shape[0], np.float64)
    lib().orc_lb2(_p(qpaa), _p(sym), sym.shape[0], sym.shape[1], L, _p(beta), _p(out))
    return out
