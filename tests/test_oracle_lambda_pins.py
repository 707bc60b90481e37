"""Pins of the oracle's factorization partition lambda(f) (Sec. 1.1, eq. 1.2).

The oracle finds lambda by distinct-degree factorization.  Here it is checked
against (i) trial division by every monic polynomial of small degree, in
table-built field models that share nothing with the oracle, and (ii) the
closed count of square-free polynomials by factorization type: over F_q there
are I_j = (1/j) sum_{d | j} mu(d) q^(j/d) monic irreducible polynomials of
degree j (Gauss), so exactly (q - 1) prod_j C(I_j, n_j) square-free
polynomials of degree sum_j j n_j have n_j irreducible factors of degree j.
"""
from __future__ import annotations

import collections
import itertools
import math

import numpy as np
import pytest

from fieldmodels import TableField, prime_power_model


def _mobius(n):
    r, m, p = 1, n, 2
    while p * p <= m:
        if m % p == 0:
            m //= p
            if m % p == 0:
                return 0
            r = -r
        p += 1
    return -r if m > 1 else r


def _irreducible_count(q, j):
    return sum(_mobius(d) * q ** (j // d) for d in range(1, j + 1) if j % d == 0) // j


# --- polynomial arithmetic over a TableField (coefficient lists, low first) ---

class _Poly:
    def __init__(self, F: TableField):
        self.F = F
        Q = F.Q
        self.inv = np.zeros(Q, dtype=np.int64)
        for a in range(1, Q):
            self.inv[a] = int(np.nonzero(F.mul[a] == 1)[0][0])

    def trim(self, a):
        a = list(a)
        while a and a[-1] == 0:
            a.pop()
        return a

    def divmod(self, a, b):
        F = self.F
        a = self.trim(a)
        b = self.trim(b)
        qt = [0] * max(len(a) - len(b) + 1, 1)
        ib = self.inv[b[-1]]
        while len(a) >= len(b):
            s = len(a) - len(b)
            f = F.mul[a[-1], ib]
            qt[s] = int(f)
            for i, c in enumerate(b):
                a[s + i] = int(F.add[a[s + i], F.neg[F.mul[f, c]]])
            a = self.trim(a)
        return self.trim(qt), a


def _factor_type(P: _Poly, coeffs, g):
    """Degrees of the irreducible factors by trial division with every monic
    polynomial of degree 1, 2, ... (a divisor found at the smallest degree is
    irreducible), plus the part 1 at infinity for odd degree."""
    F = P.F
    f = P.trim(coeffs)
    d = len(f) - 1
    mult = collections.Counter()
    if d == 2 * g + 1:
        mult[1] += 1
    k = 1
    while len(f) - 1 >= 2 * k:
        found = False
        for tail in itertools.product(range(F.Q), repeat=k):
            h = list(tail) + [1]
            qt, r = P.divmod(f, h)
            if not r:
                mult[k] += 1
                f = qt
                found = True
                break
        if not found:
            k += 1
    if len(f) - 1 > 0:
        mult[len(f) - 1] += 1
    return mult


def _as_rows(mults, g):
    out = np.zeros((len(mults), 2 * g + 2), dtype=np.uint8)
    for i, m in enumerate(mults):
        for j, c in m.items():
            out[i, j - 1] = c
    return out


def test_partitions_sum_to_2g_plus_2(oracle_mod, curvegen_mod):
    for q, g in ((3, 1), (5, 2), (13, 3), (7, 4), (9, 2), (27, 1)):
        c = curvegen_mod.sample(q, g, 200, seed=7)
        lam = oracle_mod.factor_degrees(q, g, c).astype(np.int64)
        assert ((lam * np.arange(1, 2 * g + 3)).sum(axis=1) == 2 * g + 2).all(), (q, g)


@pytest.mark.parametrize("p,g,n", [(3, 1, 60), (3, 2, 80), (5, 2, 60), (7, 2, 40), (3, 3, 30), (5, 3, 20)])
def test_trial_division_prime_fields(oracle_mod, curvegen_mod, p, g, n):
    P = _Poly(TableField.prime(p))
    c = curvegen_mod.sample(p, g, n, seed=100 + p + g)
    want = _as_rows([_factor_type(P, [int(v) for v in row], g) for row in c], g)
    assert np.array_equal(oracle_mod.factor_degrees(p, g, c), want)


def test_trial_division_q9(oracle_mod, curvegen_mod):
    """q = 9 over the coefficient-code convention (F_3[t]/(lex-first primitive))."""
    F = prime_power_model(3, 2, oracle_mod.primitive_poly(3, 2))
    P = _Poly(F)
    c = curvegen_mod.sample(9, 2, 40, seed=9)
    want = _as_rows([_factor_type(P, [int(v) for v in row], 2) for row in c], 2)
    assert np.array_equal(oracle_mod.factor_degrees(9, 2, c), want)


@pytest.mark.parametrize("q,g", [(3, 2), (5, 2), (3, 3)])
def test_type_counts_of_full_enumeration(oracle_mod, curvegen_mod, q, g):
    """Every square-free polynomial of degree 2g+1 and 2g+2: the number with
    each factorization type is (q-1) prod_j C(I_j, n_j)."""
    c = curvegen_mod.enumerate_all(q, g)
    lam = oracle_mod.factor_degrees(q, g, c).astype(np.int64)
    odd = c[:, -1] == 0
    seen = collections.Counter()
    for row, o in zip(lam, odd):
        r = row.copy()
        if o:
            r[0] -= 1           # drop the part at infinity
        seen[(bool(o), tuple(r))] += 1
    I = [_irreducible_count(q, j) for j in range(1, 2 * g + 3)]
    for (o, r), cnt in seen.items():
        want = (q - 1) * math.prod(math.comb(I[j], r[j]) for j in range(2 * g + 2))
        assert cnt == want, (o, r, cnt, want)
    # and every type with a nonzero count occurs
    for D, o in ((2 * g + 2, False), (2 * g + 1, True)):
        total = sum(v for (oo, _), v in seen.items() if oo == o)
        assert total == (q - 1) * (q ** D - q ** (D - 1))     # square-free count of degree D
