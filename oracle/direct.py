"""ORACLE (test infrastructure only): Python loader for the plain C direct sum.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this.
``build()`` compiles ``direct.c`` with gcc into ``liboracle_direct.so`` beside it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "direct.c")
LIB = os.path.join(HERE, "liboracle_direct.so")

KERNELS = {"yukawa_ss": 0, "coulomb_ss": 1, "yukawa": 2, "coulomb": 3}

_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-pthread", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_direct.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      dp, dp, dp, dp, dp, ctypes.c_int64,
                                      dp, dp, dp, dp, ctypes.c_int64, dp, dp, ctypes.c_int]
        lib.oracle_direct.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def direct_sum(kernel: str, sx, sy, sz, sf, sw, tx=None, ty=None, tz=None, tf=None,
               kappa: float = 1.0, alpha: float = 1.0, threads: int | None = None,
               return_abs: bool = False):
    """u at the targets (default: the sources themselves) by the direct sum.

    kernel: 'yukawa_ss', 'coulomb_ss', 'yukawa' or 'coulomb'. With return_abs,
    also returns sum_j |term_ij| per target (a scale for rounding tolerances)."""
    if tx is None:
        tx, ty, tz, tf = sx, sy, sz, sf
    sx, sy, sz, sf, sw = map(_f64, (sx, sy, sz, sf, sw))
    tx, ty, tz, tf = map(_f64, (tx, ty, tz, tf))
    nt = tx.size
    out = np.empty(nt)
    ab = np.empty(nt) if return_abs else None
    rc = _load().oracle_direct(KERNELS[kernel], float(kappa), float(alpha),
                               _ptr(sx), _ptr(sy), _ptr(sz), _ptr(sf), _ptr(sw), sx.size,
                               _ptr(tx), _ptr(ty), _ptr(tz), _ptr(tf), nt, _ptr(out), _ptr(ab),
                               threads or default_threads())
    if rc != 0:
        raise ValueError("oracle_direct rejected its arguments")
    return (out, ab) if return_abs else out
