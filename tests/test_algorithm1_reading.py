"""The reading of Algorithm 1's reduced enumeration (Sec. 1.2-1.3), checked on
the CPU with the oracle: every class of twist-reduced representatives,
weighted by its multiplicity and entered for f and for its quadratic twist,
reproduces the map N_{g,q} of eq. (1.2) taken over the full enumeration.

The classes follow the reading the library implements: for p not dividing d,
a translation makes c_{d-1} = 0, i is the highest nonzero position below d
and j the next one (or none), c_i = 1, c_j runs over representatives of
F_q^x / F_q^x(i-j), lower positions are free, and the multiplicity is
q (q-1)^2 / (2 gcd(q-1, i-j)) (q (q-1) / 2 without j); for p dividing d only
the scalings are used (i up to d-1, multiplicities without the factor q).
The twist's invariants follow from a_k(nf) = (-1)^k a_k(f).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest

from fieldmodels import TableField, prime_power_model


def _generator_codes(q, oracle_mod):
    """Powers 1, w, w^2, .. of a generator w of F_q^x, as codes."""
    p = next(f for f in range(3, q + 1, 2) if q % f == 0)
    e = round(math.log(q, p))
    F = TableField.prime(p) if e == 1 else prime_power_model(p, e, oracle_mod.primitive_poly(p, e))
    for w in range(2, q):
        seq, v = [1], w
        while v != 1:
            seq.append(int(v))
            v = F.mul[v, w]
        if len(seq) == q - 1:
            return seq, p
    raise AssertionError("no generator")


def _classes(q, p, g, pw):
    qm = q - 1
    for d in (2 * g + 1, 2 * g + 2):
        trans = d % p != 0
        imax = d - 2 if trans else d - 1
        for i in range(imax + 1):
            yield d, i, -1, [], (q * qm // 2 if trans else qm // 2)
            for j in range(i):
                gk = math.gcd(qm, i - j)
                yield d, i, j, pw[:gk], (q if trans else 1) * qm * qm // (2 * gk)


def _rows(q, g, d, i, j, cj):
    out = []
    for cd in range(1, q):
        for c in (cj if j >= 0 else [None]):
            for free in itertools.product(range(q), repeat=max(j, 0)):
                r = [0] * (2 * g + 3)
                r[:len(free)] = free
                if j >= 0:
                    r[j] = c
                r[i] = 1
                r[d] = cd
                out.append(r)
    return np.array(out, dtype=np.int16)


def _key(q, g, N, lam_row):
    from paper_1805_11991_amd import hwcount
    return tuple(q ** (k + 1) + 1 - int(N[k]) for k in range(g)) + (hwcount.lambda_code(lam_row),)


@pytest.mark.parametrize("q,g", [(3, 1), (5, 1), (7, 1), (9, 1), (3, 2), (5, 2), (3, 3)])
def test_reduced_enumeration_reproduces_full_map(oracle_mod, curvegen_mod, q, g):
    pw, p = _generator_codes(q, oracle_mod)
    acc = {}
    for d, i, j, cj, mult in _classes(q, p, g, pw):
        rows = _rows(q, g, d, i, j, cj)
        rows = rows[np.array([curvegen_mod.is_squarefree(q, r) for r in rows], dtype=bool)]
        if not len(rows):
            continue
        N = oracle_mod.count_curves(q, g, rows)
        lam = oracle_mod.factor_degrees(q, g, rows)
        for Nr, lr in zip(N, lam):
            Nt = [2 * (q ** (k + 1) + 1) - int(Nr[k]) if k % 2 == 0 else int(Nr[k]) for k in range(g)]
            for NN in (Nr, Nt):
                kk = _key(q, g, NN, lr)
                acc[kk] = acc.get(kk, 0) + mult
    full = curvegen_mod.enumerate_all(q, g)
    ref = {}
    for Nr, lr in zip(oracle_mod.count_curves(q, g, full), oracle_mod.factor_degrees(q, g, full)):
        kk = _key(q, g, Nr, lr)
        ref[kk] = ref.get(kk, 0) + 1
    assert acc == ref
