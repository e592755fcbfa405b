"""CPU oracle for the matrix profile: plain FP64 brute force (oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never does. It shares no code with
the GPU path. See oracle.c for what is computed and which passage of the paper
each part follows.

Parity: pinned by the CPU tests in tests/test_oracle_*.py (library routines,
exact integer brute force, the Pearson closed form of Lemma 3, the paper's
incremental algorithms, invariants, special cases and the golden fixtures).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EUCLID, PNORM, ZNORM = 0, 1, 2
KINDS = {"aamp": EUCLID, "euclid": EUCLID, "pnorm": PNORM, "acamp": ZNORM, "znorm": ZNORM}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                        "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _bind(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(ctypes.c_int64)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.oracle_profile.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_double, ctypes.c_int32, lp, ctypes.c_int64,
                                   dp, lp, dp, ctypes.c_int32]
    lib.oracle_profile.restype = ctypes.c_int
    lib.oracle_profile_diagonals.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_double, ctypes.c_int32, u8p, lp,
                                             ctypes.c_int64, dp, lp, dp, ctypes.c_int32]
    lib.oracle_profile_diagonals.restype = ctypes.c_int
    lib.oracle_window_stats.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, dp, dp, u8p]
    lib.oracle_window_stats.restype = ctypes.c_int
    lib.oracle_distance.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_double, ctypes.c_int64, ctypes.c_int64]
    lib.oracle_distance.restype = ctypes.c_double
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _lptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _kind(kind) -> int:
    return KINDS[kind] if isinstance(kind, str) else int(kind)


def profile(T, m: int, kind="aamp", p: float = 2.0, excl: int = 1, rows=None,
            nthreads: int = 0, diagonals=None):
    """Matrix profile by brute force. Returns (P, I, Q) as numpy arrays,
    one entry per row in ``rows`` (all N rows when rows is None).

    ``diagonals``: optional boolean mask of N entries; only pairs whose
    diagonal |i - j| is marked are candidates (the profile an anytime sweep
    has after visiting exactly those diagonals)."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    n = T.shape[0]
    N = n - m + 1
    if rows is None:
        R = N
        rows_arr = None
    else:
        rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        R = rows_arr.shape[0]
    P = np.empty(max(R, 0), dtype=np.float64)
    I = np.empty(max(R, 0), dtype=np.int64)
    Q = np.empty(max(R, 0), dtype=np.float64)
    rows_p = _lptr(rows_arr) if rows_arr is not None else None
    if diagonals is None:
        rc = _load().oracle_profile(_dptr(T), n, m, _kind(kind), float(p), int(excl), rows_p, R,
                                    _dptr(P), _lptr(I), _dptr(Q), int(nthreads))
    else:
        mask = np.ascontiguousarray(diagonals, dtype=np.uint8)
        if mask.shape != (max(N, 0),):
            raise ValueError("diagonals must hold one entry per window")
        rc = _load().oracle_profile_diagonals(
            _dptr(T), n, m, _kind(kind), float(p), int(excl),
            mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), rows_p, R,
            _dptr(P), _lptr(I), _dptr(Q), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_profile rejected its arguments (rc={rc})")
    return P, I, Q


def window_stats(T, m: int):
    """(mu, sigma, isconst) of every length-m window (two-pass, population)."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    N = T.shape[0] - m + 1
    mu = np.empty(N)
    sg = np.empty(N)
    c = np.empty(N, dtype=np.uint8)
    rc = _load().oracle_window_stats(_dptr(T), T.shape[0], m, _dptr(mu), _dptr(sg),
                                     c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc != 0:
        raise ValueError("oracle_window_stats rejected its arguments")
    return mu, sg, c.astype(bool)


def distance(T, m: int, i: int, j: int, kind="aamp", p: float = 2.0) -> float:
    """Distance of one pair, straight from the definition."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    return float(_load().oracle_distance(_dptr(T), T.shape[0], m, _kind(kind), float(p),
                                         int(i), int(j)))


def num_threads() -> int:
    return int(_load().oracle_num_threads())
