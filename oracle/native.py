"""Loader for the brute-force FP64 C kernels in ``hitref.c``.

Test infrastructure: see the package docstring.  ``build()`` compiles the C
file with gcc (no GPU code involved); ``closest_hit`` and ``occluded`` wrap
the two entry points with float64 NumPy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hitref.c")
_LIB = os.path.join(_HERE, "_hitref.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, f64, i32 = ctypes.c_int64, ctypes.c_double, ctypes.c_int
        lib.oracle_closest_hit.argtypes = [i64, P, P, P, f64, i64, P, i64, P, P, P, P, P, i32]
        lib.oracle_closest_hit.restype = None
        lib.oracle_segments_occluded.argtypes = [i64, P, P, P, P, f64, i64, P, i64, P, P, P, i32]
        lib.oracle_segments_occluded.restype = None
        _lib = lib
    return _lib


def default_threads() -> int:
    env = os.environ.get("ORACLE_THREADS")
    if env:
        return max(1, int(env))
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def closest_hit(O, D, excl, tmin, V, F, face, want_margin=False, threads=None):
    """Nearest triangle hit per ray (index or -1), its t, and optionally the
    edge margin (see hitref.c)."""
    lib = _load()
    O = np.ascontiguousarray(O, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.float64)
    excl = np.ascontiguousarray(excl, dtype=np.int32)
    V = np.ascontiguousarray(V, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    face = np.ascontiguousarray(face, dtype=np.int32)
    n = O.shape[0]
    tri = np.empty(n, dtype=np.int32)
    t = np.empty(n, dtype=np.float64)
    margin = np.empty(n, dtype=np.float64) if want_margin else None
    lib.oracle_closest_hit(n, _p(O), _p(D), _p(excl), float(tmin), V.shape[0], _p(V), F.shape[0], _p(F),
                           _p(face), _p(tri), _p(t), _p(margin) if want_margin else None,
                           threads or default_threads())
    return (tri, t, margin) if want_margin else (tri, t)


def occluded(A, B, excl_a, excl_b, eps, V, F, face, threads=None):
    """1 where the open segment A->B crosses a triangle (faces excl_a/excl_b skipped)."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    excl_a = np.ascontiguousarray(excl_a, dtype=np.int32)
    excl_b = np.ascontiguousarray(excl_b, dtype=np.int32)
    V = np.ascontiguousarray(V, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    face = np.ascontiguousarray(face, dtype=np.int32)
    n = A.shape[0]
    out = np.zeros(n, dtype=np.uint8)
    if n:
        lib.oracle_segments_occluded(n, _p(A), _p(B), _p(excl_a), _p(excl_b), float(eps), V.shape[0], _p(V),
                                     F.shape[0], _p(F), _p(face), _p(out), threads or default_threads())
    return out.astype(bool)
