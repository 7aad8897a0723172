"""CPU oracle for all-pairs binary mutual information -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The GPU library never imports, links or calls it, and it never
imports the GPU library.

`mi_oracle.c` holds the arithmetic: a per-pair loop over the rows that counts
the four cells (n11, n10, n01, n00) in int64 and evaluates Eq. 1/Eq. 2 of the
paper in FP64 with 0 log 0 = 0; for categorical variables (codes 0 .. L-1) the
same loop counts an L_i x L_j contingency table and Eq. 1 runs over all of
its cells.  This module builds it with gcc and wraps it
with ctypes; the wrappers do argument marshalling only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mi_oracle.c")
_LIB = os.path.join(_HERE, "libmi_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile mi_oracle.c into libmi_oracle.so (gcc, OpenMP over pairs)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.mi_oracle_pairs.argtypes = [p, i64, i64, i64, i64, p, p, p, p, p, p, p]
        lib.mi_oracle_pairs.restype = ctypes.c_int
        lib.mi_oracle_all.argtypes = [p, i64, i64, i64, p, p]
        lib.mi_oracle_all.restype = ctypes.c_int
        lib.mi_oracle_colsums.argtypes = [p, i64, i64, i64, p]
        lib.mi_oracle_colsums.restype = ctypes.c_int
        lib.mi_oracle_pairs_t.argtypes = [p, i64, i64, i64, i64, p, p, p, p, p, p, p]
        lib.mi_oracle_pairs_t.restype = ctypes.c_int
        lib.mi_oracle_colsums_t.argtypes = [p, i64, i64, i64, p]
        lib.mi_oracle_colsums_t.restype = ctypes.c_int
        lib.mi_oracle_from_counts.argtypes = [i64, i64, i64, i64]
        lib.mi_oracle_from_counts.restype = ctypes.c_double
        i32 = ctypes.c_int32
        lib.mi_oracle_cat_table.argtypes = [p, i64, i64, i64, i64, i32, i32, p]
        lib.mi_oracle_cat_table.restype = ctypes.c_int
        lib.mi_oracle_cat_from_table.argtypes = [p, i32, i32]
        lib.mi_oracle_cat_from_table.restype = ctypes.c_double
        lib.mi_oracle_cat_all.argtypes = [p, i64, i64, i64, p, p]
        lib.mi_oracle_cat_all.restype = ctypes.c_int
        lib.mi_oracle_threads.argtypes = []
        lib.mi_oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _as_u8(X) -> np.ndarray:
    X = np.asarray(X)
    if X.ndim != 2:
        raise ValueError("X must be 2-D (rows x cols)")
    if X.dtype != np.uint8:
        X = X.astype(np.uint8)
    return np.ascontiguousarray(X)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def threads() -> int:
    return int(_load().mi_oracle_threads())


def all_pairs(X, n: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """(n11 int64[n, n], MI float64[n, n] in bits) for the first n columns of X."""
    X = _as_u8(X)
    m, ld = X.shape
    n = ld if n is None else n
    n11 = np.empty((n, n), dtype=np.int64)
    mi = np.empty((n, n), dtype=np.float64)
    rc = _load().mi_oracle_all(_ptr(X), m, n, ld, _ptr(n11), _ptr(mi))
    if rc != 0:
        raise ValueError(f"mi_oracle_all rc={rc}")
    return n11, mi


def pairs(X, pi, pj, n: Optional[int] = None):
    """Counts and MI for the listed pairs: dict of int64 n11/n10/n01/n00 and float64 mi."""
    X = _as_u8(X)
    m, ld = X.shape
    n = ld if n is None else n
    pi = np.ascontiguousarray(pi, dtype=np.int64)
    pj = np.ascontiguousarray(pj, dtype=np.int64)
    if pi.shape != pj.shape or pi.ndim != 1:
        raise ValueError("pi and pj must be 1-D and the same length")
    k = pi.shape[0]
    out = {name: np.empty(k, dtype=np.int64) for name in ("n11", "n10", "n01", "n00")}
    out["mi"] = np.empty(k, dtype=np.float64)
    rc = _load().mi_oracle_pairs(_ptr(X), m, n, ld, k, _ptr(pi), _ptr(pj), _ptr(out["n11"]), _ptr(out["n10"]),
                                 _ptr(out["n01"]), _ptr(out["n00"]), _ptr(out["mi"]))
    if rc != 0:
        raise ValueError(f"mi_oracle_pairs rc={rc}")
    return out


def pairs_t(Xt, pi, pj, n: Optional[int] = None):
    """pairs() on the transposed layout: Xt is (cols, m), row j holding column j's m entries."""
    Xt = _as_u8(Xt)
    ncols, m = Xt.shape
    n = ncols if n is None else n
    pi = np.ascontiguousarray(pi, dtype=np.int64)
    pj = np.ascontiguousarray(pj, dtype=np.int64)
    if pi.shape != pj.shape or pi.ndim != 1:
        raise ValueError("pi and pj must be 1-D and the same length")
    if n > ncols:
        raise ValueError("n exceeds the rows of Xt")
    k = pi.shape[0]
    out = {name: np.empty(k, dtype=np.int64) for name in ("n11", "n10", "n01", "n00")}
    out["mi"] = np.empty(k, dtype=np.float64)
    rc = _load().mi_oracle_pairs_t(_ptr(Xt), m, n, m, k, _ptr(pi), _ptr(pj), _ptr(out["n11"]), _ptr(out["n10"]),
                                   _ptr(out["n01"]), _ptr(out["n00"]), _ptr(out["mi"]))
    if rc != 0:
        raise ValueError(f"mi_oracle_pairs_t rc={rc}")
    return out


def colsums_t(Xt, n: Optional[int] = None) -> np.ndarray:
    """colsums() on the transposed layout (cols, m)."""
    Xt = _as_u8(Xt)
    ncols, m = Xt.shape
    n = ncols if n is None else n
    if n > ncols:
        raise ValueError("n exceeds the rows of Xt")
    c = np.empty(n, dtype=np.int64)
    rc = _load().mi_oracle_colsums_t(_ptr(Xt), m, n, m, _ptr(c))
    if rc != 0:
        raise ValueError(f"mi_oracle_colsums_t rc={rc}")
    return c


def colsums(X, n: Optional[int] = None) -> np.ndarray:
    X = _as_u8(X)
    m, ld = X.shape
    n = ld if n is None else n
    c = np.empty(n, dtype=np.int64)
    rc = _load().mi_oracle_colsums(_ptr(X), m, n, ld, _ptr(c))
    if rc != 0:
        raise ValueError(f"mi_oracle_colsums rc={rc}")
    return c


def from_counts(n11: int, n10: int, n01: int, n00: int) -> float:
    """MI in bits of one pair from its four cell counts (Eq. 2)."""
    return float(_load().mi_oracle_from_counts(int(n11), int(n10), int(n01), int(n00)))


def _levels(levels, v: int) -> np.ndarray:
    lv = np.ascontiguousarray(levels, dtype=np.int32)
    if lv.shape != (v,):
        raise ValueError("levels must hold one count per variable")
    return lv


def cat_table(X, levels, i: int, j: int) -> np.ndarray:
    """Contingency table (int64[L_i, L_j]) of categorical variables i and j."""
    X = _as_u8(X)
    m, ld = X.shape
    lv = np.asarray(levels, dtype=np.int64)
    Li, Lj = int(lv[i]), int(lv[j])
    t = np.empty((Li, Lj), dtype=np.int64)
    rc = _load().mi_oracle_cat_table(_ptr(X), m, ld, int(i), int(j), Li, Lj, _ptr(t))
    if rc != 0:
        raise ValueError(f"mi_oracle_cat_table rc={rc}")
    return t


def cat_from_table(table) -> float:
    """MI in bits of one pair from its contingency table (Eq. 1 over all cells)."""
    t = np.ascontiguousarray(table, dtype=np.int64)
    if t.ndim != 2:
        raise ValueError("table must be 2-D")
    return float(_load().mi_oracle_cat_from_table(_ptr(t), t.shape[0], t.shape[1]))


def cat_all_pairs(X, levels, v: Optional[int] = None) -> np.ndarray:
    """MI float64[v, v] in bits between the first v categorical columns of X,
    column j holding codes 0 .. levels[j] - 1."""
    X = _as_u8(X)
    m, ld = X.shape
    v = ld if v is None else v
    lv = _levels(levels, v)
    mi = np.empty((v, v), dtype=np.float64)
    rc = _load().mi_oracle_cat_all(_ptr(X), m, v, ld, _ptr(lv), _ptr(mi))
    if rc != 0:
        raise ValueError(f"mi_oracle_cat_all rc={rc}")
    return mi
