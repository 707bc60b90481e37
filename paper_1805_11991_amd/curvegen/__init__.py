"""Seeded synthetic curve sets (inputs only; see ``curvegen.c``).

Rows are coefficient codes a_0 .. a_{2g+2} (constant term first) of
square-free f of degree 2g+1 or 2g+2 over F_q.  int8 when q <= 127, else
int16.  Random streams are keyed by (seed, q, g) and each curve by its index,
so any slice of a stream can be regenerated on its own.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "curvegen.c")
_LIB = os.path.join(_HERE, "libcurvegen.so")
_lib = None

#: base seed of the synthetic workloads; the workload index is added to it
BASE_SEED = 180511991


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.cg_sample.restype = ctypes.c_int
        lib.cg_sample.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                  ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
        lib.cg_enumerate.restype = ctypes.c_int64
        lib.cg_enumerate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_int64]
        lib.cg_is_squarefree.restype = ctypes.c_int
        lib.cg_is_squarefree.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
        _lib = lib
    return _lib


def code_dtype(q: int):
    return np.int8 if q <= 127 else np.int16


def sample(q: int, g: int, n: int, seed: int, start: int = 0, threads: int | None = None,
           dtype=None) -> np.ndarray:
    """Curves start .. start+n-1 of the stream (seed, q, g): [n, 2g+3] codes."""
    dtype = code_dtype(q) if dtype is None else np.dtype(dtype).type
    width = 1 if dtype == np.int8 else 2
    out = np.empty((n, 2 * g + 3), dtype=dtype)
    if threads is None:
        threads = min(os.cpu_count() or 1, 16)
    if n and _load().cg_sample(seed, q, g, start, n, width, out.ctypes.data, threads) != 0:
        raise ValueError(f"cannot sample q={q} g={g}")
    return out


def enumerate_all(q: int, g: int, dtype=None) -> np.ndarray:
    """Every square-free f of degree 2g+1 or 2g+2 over F_q, in increasing
    order of sum_i a_i q^i."""
    dtype = code_dtype(q) if dtype is None else np.dtype(dtype).type
    width = 1 if dtype == np.int8 else 2
    lib = _load()
    total = lib.cg_enumerate(q, g, width, None, 0)
    if total < 0:
        raise ValueError(f"cannot enumerate q={q} g={g}")
    out = np.empty((total, 2 * g + 3), dtype=dtype)
    lib.cg_enumerate(q, g, width, out.ctypes.data, total)
    return out


def is_squarefree(q: int, codes) -> bool:
    c = np.ascontiguousarray(np.asarray(codes, dtype=np.int32))
    r = _load().cg_is_squarefree(q, c.ctypes.data, c.shape[0])
    if r < 0:
        raise ValueError("bad field")
    return bool(r)
