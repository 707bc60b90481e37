"""The C ABI library on the CPU: it loads, exports every declared symbol, and
its host-side field tables satisfy their definitions (Sec. 2.3, encoding
(3.1), table (3.2)).  No counting call runs here (that needs a GPU).

Tables are not compared to fixed values (they depend on the generator); they
are checked against invariants, using the oracle's independent polynomial
arithmetic where a product is needed.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1805_11991_amd import hwcount

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hctx():
    ctx = hwcount.Context(device=-1)
    yield ctx
    ctx.close()


def test_exports_every_declared_symbol():
    lib = hwcount.load()
    header = open(os.path.join(ROOT, "include", "hwcount.h")).read()
    declared = set(re.findall(r"\b(hwc_[a-z_]+)\s*\(", header))
    assert declared == set(hwcount.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_host_only_context_refuses_counting(hctx):
    with pytest.raises(hwcount.HwcError) as ei:
        hctx.count_curves(5, 2, np.array([[1, 0, 0, 0, 0, 1, 0]]))
    assert ei.value.code == hwcount.HWC_ERR_NO_DEVICE


def test_bad_field_arguments(hctx):
    for p, e, k in ((15, 1, 1), (2, 1, 1), (9, 1, 1)):
        with pytest.raises(hwcount.HwcError) as ei:
            hctx.build_field(p, e, k)
        assert ei.value.code == hwcount.HWC_ERR_NOT_ODD_PRIME_POWER


def _digits(v, p, n):
    return [(v // p ** i) % p for i in range(n)]


@pytest.mark.parametrize("p,e,k", [(5, 1, 1), (5, 1, 2), (13, 1, 3), (3, 2, 2), (3, 1, 4), (7, 2, 1), (5, 2, 2),
                                   (13, 1, 4)])
def test_field_tables_invariants(hctx, oracle_mod, p, e, k):
    F = hctx.build_field(p, e, k)
    info = F.info()
    n = e * k
    Q = p ** n
    M = Q - 1
    assert (info.p, info.e, info.k, info.n, info.Q, info.q) == (p, e, k, n, Q, p ** e)
    # the modulus is the lex-first primitive polynomial (same rule as the oracle's own search)
    assert list(info.modulus[:n + 1]) == oracle_mod.primitive_poly(p, n)
    T = F.tables()
    exp, log, zech, emb = T["exp"].astype(np.int64), T["log"], T["zech"], T["emb"].astype(np.int64)
    # exp walks t^L with the oracle's product; it is a bijection onto F_Q^x
    t_packed = p if n > 1 else (p - info.modulus[0]) % p
    assert exp[0] == 1
    for L in range(0, M, max(1, M // 500)):
        assert oracle_mod.field_mul(p, n, int(exp[L]), t_packed) == exp[(L + 1) % M]
    assert len(set(exp.tolist())) == M and 0 not in set(exp.tolist())
    # log inverts exp, with the zero sentinel M (encoding (3.1))
    assert log[0] == M
    assert (log[exp] == np.arange(M)).all()
    # Zech: t^Z(L) = 1 + t^L, sentinel M where 1 + t^L = 0 (table (3.2))
    plus_one = exp - exp % p + (exp % p + 1) % p
    zero = plus_one == 0
    assert zero.sum() == 1 and np.flatnonzero(zero)[0] == M // 2
    assert zech[M // 2] == M
    nz = ~zero
    assert (exp[zech[nz]] == plus_one[nz]).all()
    # Z(-L) = Z(L) - L (mod M)
    L = np.arange(1, M)
    ok = (zech[L] != M)
    assert ((zech[(M - L[ok]) % M] - (zech[L[ok]] - L[ok])) % M == 0).all()
    # emb: F_q -> F_Q is additive and multiplicative (the oracle multiplies in F_q)
    q = p ** e
    assert emb[0] == M
    for a in range(1, q):
        for b in range(1, q, max(1, q // 7)):
            ab = oracle_mod.field_mul(p, e, a, b)
            assert emb[ab] == (emb[a] + emb[b]) % M
            s = sum(((x + y) % p) * p ** i for i, (x, y) in enumerate(zip(_digits(a, p, e), _digits(b, p, e))))
            lhs = 0 if s == 0 else int(exp[emb[s]])
            rhs = sum(((x + y) % p) * p ** i for i, (x, y) in
                      enumerate(zip(_digits(int(exp[emb[a]]), p, n), _digits(int(exp[emb[b]]), p, n))))
            assert lhs == rhs
    # Frobenius orbits of size exactly k: sum_{d | k} mu(k/d) q^d elements of degree k
    def mu(m):
        r, d = 1, 2
        while d * d <= m:
            if m % d == 0:
                m //= d
                if m % d == 0:
                    return 0
                r = -r
            d += 1
        return -r if m > 1 else r
    exact = sum(mu(k // d) * q ** d for d in range(1, k + 1) if k % d == 0) - (1 if k == 1 else 0)
    reps = T["prim_reps"]
    assert len(reps) * k == exact
    for r in reps[:50]:
        orb = {(int(r) * q ** i) % M for i in range(k)}
        assert len(orb) == k and min(orb) == r
    F.release()


def test_field_cache_is_idempotent(hctx):
    a = hctx.build_field(13, 1, 2).tables()
    b = hctx.build_field(13, 1, 2).tables()
    for key in a:
        assert (a[key] == b[key]).all()


def test_field_too_large(hctx):
    with pytest.raises(hwcount.HwcError) as ei:
        hctx.build_field(3001, 1, 3)
    assert ei.value.code == hwcount.HWC_ERR_FIELD_TOO_LARGE


def test_single_hip_runtime_in_process():
    """The library binds to the HIP runtime torch already loaded: one
    libamdhip64 mapping in the process, whichever is imported first."""
    import subprocess
    import sys
    code = ("from paper_1805_11991_amd import hwcount; hwcount.load(); import torch; "
            "maps = open('/proc/self/maps').read().split('\\n'); "
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
