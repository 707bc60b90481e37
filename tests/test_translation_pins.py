"""Translation invariance, the fact the library's dense translates rest on.

x -> x + t with t in F_q permutes every F_{q^k} and keeps the degree and the
leading coefficient of f, so y^2 = f(x) and y^2 = f(x + t) have the same N_k
(Sec. 1.1) and f, f(x + t) the same factorization pattern (eq. 1.2); the
reduction of Algorithm 1 divides out the same equivalence.  Checked here on
the oracle with the translate computed independently (binomial expansion over
F_q from the oracle's field product and digit-wise addition)."""
from __future__ import annotations

from math import comb

import numpy as np
import pytest


def _add(a: int, b: int, p: int, e: int) -> int:
    r, pw = 0, 1
    for _ in range(e):
        r += ((a // pw % p + b // pw % p) % p) * pw
        pw *= p
    return r


def _translate(oracle_mod, row, t: int, p: int, e: int):
    """Coefficients of f(x + t) = sum_i c_i (x + t)^i by the binomial theorem."""
    n = len(row)
    out = [0] * n
    tp = [1] * n                        # t^j
    for j in range(1, n):
        tp[j] = oracle_mod.field_mul(p, e, tp[j - 1], t)
    for i, c in enumerate(row):
        c = int(c)
        if c == 0:
            continue
        for k in range(i + 1):
            b = comb(i, k) % p          # integer multiple: repeated addition
            term = oracle_mod.field_mul(p, e, c, tp[i - k])
            acc = 0
            for _ in range(b):
                acc = _add(acc, term, p, e)
            out[k] = _add(out[k], acc, p, e)
    return out


@pytest.mark.parametrize("q,p,e,g", [(5, 5, 1, 2), (9, 3, 2, 2), (13, 13, 1, 3), (27, 3, 3, 2), (7, 7, 1, 4)])
def test_counts_and_partitions_are_translation_invariant(oracle_mod, curvegen_mod, q, p, e, g):
    rng = np.random.default_rng(q * 10 + g)
    rows = curvegen_mod.sample(q, g, 60, seed=4242 + q).astype(np.int64)
    # many zero coefficients below the top, as in the sparse rows translated on the GPU
    low = rng.random((rows.shape[0], rows.shape[1] - 2)) < 0.3
    rows[:, :-2][low] = 0
    shifted = np.array([_translate(oracle_mod, r, int(rng.integers(1, q)), p, e) for r in rows], dtype=np.int64)
    assert (shifted[:, -1] == rows[:, -1]).all() and (shifted[:, -2][rows[:, -1] == 0] == rows[:, -2][rows[:, -1] == 0]).all()
    assert np.array_equal(oracle_mod.count_curves(q, g, rows), oracle_mod.count_curves(q, g, shifted))
    assert np.array_equal(oracle_mod.factor_degrees(q, g, rows), oracle_mod.factor_degrees(q, g, shifted))


def test_translate_of_a_power_is_binomial(oracle_mod):
    # (x + t)^4 over F_7: coefficients C(4, k) t^(4-k) mod 7, from the closed form
    t = 3
    got = _translate(oracle_mod, [0, 0, 0, 0, 1], t, 7, 1)
    assert got == [comb(4, k) * t ** (4 - k) % 7 for k in range(5)]
