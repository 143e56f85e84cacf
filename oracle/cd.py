"""Oracle (test infrastructure only): ctypes wrapper of ``cd_plain.c``.

The shared object is built by :func:`build` (gcc, plain C) next to this file;
``__graft_entry__.build`` calls it so that the checker is compiled with the
rest of the repository. If it is missing, :func:`_lib` builds it on first use.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cd_plain.c")
_SO = os.path.join(_HERE, "liboracle_cd.so")
_handle = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _handle
    if _handle is None:
        if not os.path.exists(_SO):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        f = lib.oracle_cd_sweeps
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        f.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ip, dp, dp, ctypes.c_double,
                      ctypes.c_int, ctypes.c_double, dp, dp, dp, ctypes.c_int]
        f.restype = ctypes.c_int
        _handle = lib
    return _handle


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def cd_sweeps(W: np.ndarray, ri, ci, S_vals, A_vals, lam: float, max_sweeps: int,
              tol: float, D0=None, verbose: bool = False):
    """Cyclic CD over coordinates (ri[t], ci[t]) (local indices into W).

    Returns (Delta per coordinate, sweeps run, last sweep's max |mu|).
    verbose: a progress line per sweep on stderr.
    """
    W = np.ascontiguousarray(W, dtype=np.float64)
    nj = W.shape[0]
    ri = np.ascontiguousarray(ri, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    S_vals = np.ascontiguousarray(S_vals, dtype=np.float64)
    A_vals = np.ascontiguousarray(A_vals, dtype=np.float64)
    nc = ri.size
    D = np.zeros(nc) if D0 is None else np.array(D0, dtype=np.float64, copy=True)
    U = np.empty((nj, nj), dtype=np.float64)
    last = ctypes.c_double(0.0)
    sweeps = _lib().oracle_cd_sweeps(
        nj, _p(W, ctypes.c_double), nc, _p(ri, ctypes.c_int), _p(ci, ctypes.c_int),
        _p(S_vals, ctypes.c_double), _p(A_vals, ctypes.c_double), float(lam),
        int(max_sweeps), float(tol), _p(D, ctypes.c_double), _p(U, ctypes.c_double),
        ctypes.byref(last), int(bool(verbose)))
    return D, sweeps, last.value
