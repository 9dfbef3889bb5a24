"""ctypes wrapper of the oracle's C direct sum (test infrastructure).

``build()`` compiles ``pairsum.c`` with gcc -O2 -fopenmp into
``oracle/_pairsum.so``; ``pairsum`` calls it.  The C loop is checked in the
tests against the dense NumPy blocks of ``kernels.dense_block``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pairsum.c")
_LIB = os.path.join(_HERE, "_pairsum.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        f = lib.oracle_pairsum
        P = ctypes.c_void_p
        f.argtypes = [ctypes.c_int64, P, P, ctypes.c_int64, P, P, P, P,
                      ctypes.c_double, ctypes.c_int, P]
        f.restype = None
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def pairsum(x, y, kinds, lam, mu, tsph=None, ssph=None, skip_same=False):
    """u (nt x 3) = sum_j K_j(x_i - y_j) lam_j, optionally skipping pairs in
    the same sphere."""
    lib = _load()
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    lam = np.ascontiguousarray(np.reshape(lam, (-1, 3)), np.float64)
    kinds = np.ascontiguousarray(kinds, np.int32)
    nt, ns = x.shape[0], y.shape[0]
    if skip_same:
        tsph = np.ascontiguousarray(tsph, np.int32)
        ssph = np.ascontiguousarray(ssph, np.int32)
    else:
        tsph = None
        ssph = np.zeros(ns, np.int32)
    u = np.zeros((nt, 3))
    if nt and ns:
        lib.oracle_pairsum(nt, _p(x), _p(tsph), ns, _p(y), _p(kinds), _p(ssph),
                           _p(lam), float(mu), int(bool(skip_same)), _p(u))
    return u
