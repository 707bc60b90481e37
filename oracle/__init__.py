"""CPU reference for the curve counts -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The library path in
``paper_1805_11991_amd`` never imports it and shares no code with it.

The counting itself lives in ``hwc_oracle.c`` (plain C, polynomial-basis
arithmetic, see its header).  This module compiles it with gcc and wraps it
with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hwc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (gcc, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    lib.orc_count_curves.restype = ctypes.c_int
    lib.orc_count_curves.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.orc_primitive_poly.restype = ctypes.c_int
    lib.orc_primitive_poly.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    lib.orc_square_table.restype = ctypes.c_int
    lib.orc_square_table.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    lib.orc_field_mul.restype = ctypes.c_int64
    lib.orc_field_mul.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64]
    lib.orc_factor_degrees.restype = ctypes.c_int
    lib.orc_factor_degrees.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_int]
    lib.orc_histogram.restype = ctypes.c_int64
    lib.orc_histogram.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_int64]
    _lib = lib
    return lib


def count_curves(q: int, g: int, codes, kmax: int | None = None, threads: int | None = None,
                 modulus_last: bool = False, root_last: bool = False) -> np.ndarray:
    """N_k for k = 1..kmax (default g) for every row of ``codes`` ([n, 2g+3],
    constant term first).  Returns int32 [n, kmax]."""
    lib = _load()
    c = np.ascontiguousarray(np.asarray(codes), dtype=np.int16)
    if c.ndim != 2 or c.shape[1] != 2 * g + 3:
        raise ValueError(f"codes must be [n, {2 * g + 3}]")
    kmax = g if kmax is None else kmax
    n = c.shape[0]
    out = np.zeros((n, kmax), dtype=np.int32)
    if threads is None:
        threads = min(os.cpu_count() or 1, 16)
    variant = (1 if modulus_last else 0) | (2 if root_last else 0)
    rc = lib.orc_count_curves(q, g, kmax, c.ctypes.data, n, out.ctypes.data, threads, variant)
    if rc != 0:
        raise ValueError(f"oracle rejected input (code {rc})")
    return out


def factor_degrees(q: int, g: int, codes, threads: int | None = None) -> np.ndarray:
    """lambda(f) of every row (Sec. 1.1): uint8 [n, 2g+2], entry j-1 = number of
    irreducible factors of degree j over F_q, with the extra part 1 of an odd
    degree row counted in column 0.  Distinct-degree factorization in plain
    polynomial arithmetic."""
    lib = _load()
    c = np.ascontiguousarray(np.asarray(codes), dtype=np.int16)
    if c.ndim != 2 or c.shape[1] != 2 * g + 3:
        raise ValueError(f"codes must be [n, {2 * g + 3}]")
    n = c.shape[0]
    out = np.zeros((n, 2 * g + 2), dtype=np.uint8)
    if threads is None:
        threads = min(os.cpu_count() or 1, 16)
    rc = lib.orc_factor_degrees(q, g, c.ctypes.data, n, out.ctypes.data, threads)
    if rc != 0:
        raise ValueError(f"oracle rejected input (code {rc})")
    return out


def primitive_poly(p: int, n: int, last: bool = False) -> list[int]:
    """Lex-first (or lex-last) primitive monic polynomial of degree n over F_p,
    coefficients constant term first (last entry 1)."""
    out = np.zeros(n + 1, dtype=np.int32)
    if _load().orc_primitive_poly(p, n, 1 if last else 0, out.ctypes.data) != 0:
        raise ValueError("no primitive polynomial")
    return [int(v) for v in out]


def square_table(p: int, n: int) -> np.ndarray:
    """uint8[p^n]: 1 where the packed element is a nonzero square."""
    out = np.zeros(p ** n, dtype=np.uint8)
    if _load().orc_square_table(p, n, out.ctypes.data) != 0:
        raise ValueError("bad field")
    return out


def field_mul(p: int, n: int, a: int, b: int) -> int:
    return int(_load().orc_field_mul(p, n, a, b))


def histogram(N: np.ndarray):
    """Distinct rows of N in lexicographic order and their multiplicities."""
    lib = _load()
    N = np.ascontiguousarray(N, dtype=np.int32)
    n, w = N.shape
    keys = np.zeros((max(n, 1), w), dtype=np.int32)
    counts = np.zeros(max(n, 1), dtype=np.uint64)
    d = lib.orc_histogram(N.ctypes.data, n, w, keys.ctypes.data, counts.ctypes.data, n)
    if d < 0:
        raise MemoryError
    return keys[:d].copy(), counts[:d].copy()
