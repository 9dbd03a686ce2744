"""Loader for the plain C Slater-Condon apply (oracle/sc_apply.c).

TEST INFRASTRUCTURE ONLY.  Compiles the C file with gcc into
``oracle/_build/liboracle_sc.so`` on first use (or when the source is newer)
and calls it through ctypes.  IEEE semantics are kept (-O2, no fast-math).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc_apply.c")
_OUT = os.path.join(_HERE, "_build", "liboracle_sc.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc, OpenMP).  Returns the library path."""
    os.makedirs(os.path.dirname(_OUT), exist_ok=True)
    if force or not os.path.exists(_OUT) or os.path.getmtime(_OUT) < os.path.getmtime(_SRC):
        tmp = _OUT + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                        "-o", tmp, _SRC], check=True)
        os.replace(tmp, _OUT)
    return _OUT


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            lib.oracle_sc_apply.restype = None
            lib.oracle_sc_apply.argtypes = [
                ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                ctypes.c_int64]
            _lib = lib
    return _lib


def apply(n: int, h: np.ndarray, g: np.ndarray, keys: np.ndarray, w: np.ndarray,
          rows: np.ndarray | None = None) -> np.ndarray:
    """u = H w (all rows) or u[k] = (H w)[rows[k]]."""
    lib = _load()
    h = np.ascontiguousarray(h, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    assert h.shape == (n, n) and g.shape == (n, n, n, n) and w.shape == keys.shape
    if rows is None:
        u = np.empty(keys.size, dtype=np.float64)
        lib.oracle_sc_apply(n, h.ctypes.data, g.ctypes.data, keys.ctypes.data, keys.size,
                            w.ctypes.data, u.ctypes.data, None, 0)
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        assert rows.size == 0 or (rows.min() >= 0 and rows.max() < keys.size)
        u = np.empty(rows.size, dtype=np.float64)
        lib.oracle_sc_apply(n, h.ctypes.data, g.ctypes.data, keys.ctypes.data, keys.size,
                            w.ctypes.data, u.ctypes.data, rows.ctypes.data, rows.size)
    return u


class Operator:
    """Matrix-free H on a determinant set, for use as ``H @ w``."""

    def __init__(self, n, h, g, keys):
        self.n, self.h, self.g = n, h, g
        self.keys = np.ascontiguousarray(keys, dtype=np.uint64)
        self.shape = (self.keys.size, self.keys.size)

    def __matmul__(self, w):
        w = np.asarray(w, dtype=np.float64)
        if w.ndim == 1:
            return apply(self.n, self.h, self.g, self.keys, w)
        return np.stack([apply(self.n, self.h, self.g, self.keys, w[:, j])
                         for j in range(w.shape[1])], axis=1)


def csr(n: int, h: np.ndarray, g: np.ndarray, keys: np.ndarray):
    """Hamiltonian projected on the set as scipy CSR, row by row through the C
    rules (same elements as ``hamiltonian.build``)."""
    import scipy.sparse as sp
    lib = _load()
    if not hasattr(lib, "_row_ready"):
        lib.oracle_sc_row.restype = ctypes.c_int64
        lib.oracle_sc_row.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        lib._row_ready = True
    h = np.ascontiguousarray(h, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    cap = 1 << 17
    cols = np.empty(cap, dtype=np.int64)
    vals = np.empty(cap, dtype=np.float64)
    indptr = [0]
    all_c, all_v = [], []
    for r in range(keys.size):
        c = lib.oracle_sc_row(n, h.ctypes.data, g.ctypes.data, keys.ctypes.data, keys.size, r,
                              cols.ctypes.data, vals.ctypes.data, cap)
        assert c <= cap
        order = np.argsort(cols[:c], kind="stable")
        all_c.append(cols[:c][order].copy())
        all_v.append(vals[:c][order].copy())
        indptr.append(indptr[-1] + c)
    return sp.csr_matrix((np.concatenate(all_v), np.concatenate(all_c), np.array(indptr)),
                         shape=(keys.size, keys.size))
