"""Pins of the CPU oracle against facts fixed outside it (CPU only).

The paper prints no point counts (its Table 1 holds run times), so every pin
here comes from mathematics: brute-force pair counting in independently built
field models, closed forms, the Weil bound, the quadratic-twist relation in
its corrected form, the L-polynomial, GL_2 x F_q^x invariance (Sec. 1.2) and
independence of the field model.  Each pin is chosen so that a plausible
mistake in the oracle (a dropped term at infinity, the character of the wrong
field, a wrong embedding of F_q, a transposed Horner step) fails it.
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

from fieldmodels import TableField, prime_power_model

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                yield [int(v) for v in line.split()]


def _random_curves(curvegen, q, g, n, seed=12345):
    return curvegen.sample(q, g, n, seed=seed, dtype=np.int16)


# ---------------------------------------------------------------- fields --

def test_primitive_polynomials_hand_derived(oracle_mod):
    for row in _rows("primitive_polynomials.txt"):
        p, n, coeffs = row[0], row[1], row[2:]
        assert oracle_mod.primitive_poly(p, n) == coeffs, (p, n)


def test_degree_one_primitive_root_is_textbook(oracle_mod):
    # t + a_0 is primitive iff -a_0 generates F_p^x; the first such a_0 wins
    for p in (3, 5, 7, 11, 13, 17, 19, 23, 29, 31):
        def order(r):
            k, v = 1, r % p
            while v != 1:
                v = v * r % p
                k += 1
            return k
        a0 = next(a for a in range(1, p) if order((-a) % p) == p - 1)
        assert oracle_mod.primitive_poly(p, 1) == [a0, 1]


def test_square_table_matches_jacobi_symbol(oracle_mod):
    def jacobi(a, n):
        a %= n
        res = 1
        while a:
            while a % 2 == 0:
                a //= 2
                if n % 8 in (3, 5):
                    res = -res
            a, n = n, a
            if a % 4 == 3 and n % 4 == 3:
                res = -res
            a %= n
        return res if n == 1 else 0
    for p in (3, 5, 7, 13, 31, 101):
        sq = oracle_mod.square_table(p, 1)
        # in F_p the packed value of a residue is the residue itself
        expect = np.array([1 if (v and jacobi(v, p) == 1) else 0 for v in range(p)], dtype=np.uint8)
        assert (sq == expect).all(), p


def test_square_table_euler_criterion(oracle_mod):
    for p, n in ((3, 2), (5, 2), (3, 3), (7, 2)):
        Q = p ** n
        sq = oracle_mod.square_table(p, n)
        for v in range(1, Q):
            # y^{(Q-1)/2} by repeated squaring with the oracle's product
            e, base, acc = (Q - 1) // 2, v, 1
            while e:
                if e & 1:
                    acc = oracle_mod.field_mul(p, n, acc, base)
                base = oracle_mod.field_mul(p, n, base, base)
                e >>= 1
            assert (acc == 1) == bool(sq[v]), (p, n, v)
        assert sq[0] == 0 and int(sq.sum()) == (Q - 1) // 2


# ----------------------------------------------------------- brute force --

@pytest.mark.parametrize("p", [3, 5, 7, 13])
@pytest.mark.parametrize("g", [1, 2, 3])
def test_brute_force_prime_field_k1_k2(oracle_mod, curvegen_mod, p, g):
    Fp = TableField.prime(p)
    Fp2, _ = Fp.extend(2)     # F_p[s]/(s^2 + h1 s + h0), not the oracle's model
    curves = _random_curves(curvegen_mod, p, g, 24, seed=7 + p + 10 * g)
    N = oracle_mod.count_curves(p, g, curves, kmax=2, threads=2)
    for row, n in zip(curves, N):
        c = [int(v) for v in row]
        assert Fp.count_points(c, g) == n[0]
        assert Fp2.count_points(c, g) == n[1]


@pytest.mark.parametrize("p", [3, 5])
def test_brute_force_prime_field_k3(oracle_mod, curvegen_mod, p):
    g = 2
    Fp = TableField.prime(p)
    Fp3, _ = Fp.extend(3)
    curves = _random_curves(curvegen_mod, p, g, 12, seed=99 + p)
    N = oracle_mod.count_curves(p, g, curves, kmax=3, threads=2)
    for row, n in zip(curves, N):
        assert Fp3.count_points([int(v) for v in row], g) == n[2]


def test_brute_force_prime_power_coefficients(oracle_mod, curvegen_mod):
    # q = 9: codes are d0 + 3 d1 <-> d0 + d1 t in F_3[t]/(t^2 + t + 2), the
    # hand-derived lex-first primitive polynomial.  F_81 is built over that F_9
    # by an irreducible quadratic in a second variable.
    P9 = next(r[2:] for r in _rows("primitive_polynomials.txt") if r[:2] == [3, 2])
    F9 = prime_power_model(3, 2, P9)
    F81, _ = F9.extend(2)
    for g in (1, 2):
        curves = _random_curves(curvegen_mod, 9, g, 16, seed=31 + g)
        N = oracle_mod.count_curves(9, g, curves, kmax=2, threads=2)
        for row, n in zip(curves, N):
            c = [int(v) for v in row]
            assert F9.count_points(c, g) == n[0]
            assert F81.count_points(c, g) == n[1]


def test_brute_force_q25(oracle_mod, curvegen_mod):
    P25 = next(r[2:] for r in _rows("primitive_polynomials.txt") if r[:2] == [5, 2])
    F25 = prime_power_model(5, 2, P25)
    curves = _random_curves(curvegen_mod, 25, 2, 12, seed=5)
    N = oracle_mod.count_curves(25, 2, curves, kmax=1, threads=2)
    for row, n in zip(curves, N):
        assert F25.count_points([int(v) for v in row], 2) == n[0]


# ----------------------------------------------------------- closed forms --

def test_closed_form_odd_power(oracle_mod):
    for q, g, c, k, expect in _rows("closed_forms.txt"):
        row = np.zeros((1, 2 * g + 3), dtype=np.int16)
        row[0, 0] = c
        row[0, 2 * g + 1] = 1
        assert oracle_mod.count_curves(q, g, row, kmax=k)[0, k - 1] == expect


def test_supersingular_genus_one(oracle_mod):
    for p, expect in _rows("supersingular_g1.txt"):
        row = np.array([[0, 1, 0, 1, 0]], dtype=np.int16)
        assert oracle_mod.count_curves(p, 1, row, kmax=1)[0, 0] == expect


# -------------------------------------------------------------- invariants --

def _l_poly(q, g, N):
    """b_0..b_{2g} of L(T) from N_1..N_g (Newton's identities), exact."""
    s = [None] + [q ** k + 1 - int(N[k - 1]) for k in range(1, g + 1)]
    b = [1] + [0] * (2 * g)
    for k in range(1, g + 1):
        acc = -sum(s[i] * b[k - i] for i in range(1, k + 1))
        assert acc % k == 0
        b[k] = acc // k
    for i in range(g):
        b[2 * g - i] = q ** (g - i) * b[i]
    return b, s


@pytest.mark.parametrize("q,g", [(3, 1), (3, 2), (5, 2), (3, 3), (7, 2), (9, 1), (5, 3)])
def test_weil_lpoly_next_count_and_jacobian(oracle_mod, curvegen_mod, q, g):
    n = 16 if q ** (g + 1) <= 4096 else 6
    curves = _random_curves(curvegen_mod, q, g, n, seed=1000 + q * 10 + g)
    N = oracle_mod.count_curves(q, g, curves, kmax=g + 1, threads=4)
    for row in N:
        for k in range(1, g + 2):
            dev = int(row[k - 1]) - q ** k - 1
            assert dev * dev <= 4 * g * g * q ** k, (q, g, k, row)
        b, s = _l_poly(q, g, row[:g])
        s_next = -((g + 1) * b[g + 1] + sum(s[i] * b[g + 1 - i] for i in range(1, g + 1)))
        assert row[g] == q ** (g + 1) + 1 - s_next, (q, g, row)
        assert sum(b) > 0          # L(1) = #Jac(F_q)


def _nonsquare(q):
    return next(a for a in range(2, q) if pow(a, (q - 1) // 2, q) == q - 1)


@pytest.mark.parametrize("q,g", [(5, 2), (7, 2), (13, 3), (11, 1)])
def test_quadratic_twist(oracle_mod, curvegen_mod, q, g):
    # N_k(f) + N_k(n f) = 2 (q^k + 1) for k odd, N_k(n f) = N_k(f) for k even
    curves = _random_curves(curvegen_mod, q, g, 20, seed=77 + q)
    nf = (curves.astype(np.int64) * _nonsquare(q)) % q
    kmax = 3 if q ** 3 <= 2197 else 2
    A = oracle_mod.count_curves(q, g, curves, kmax=kmax)
    B = oracle_mod.count_curves(q, g, nf.astype(np.int16), kmax=kmax)
    for k in range(1, kmax + 1):
        if k % 2:
            assert (A[:, k - 1] + B[:, k - 1] == 2 * (q ** k + 1)).all()
        else:
            assert (A[:, k - 1] == B[:, k - 1]).all()


def test_twist_as_printed_fails(oracle_mod, curvegen_mod):
    # the printed relation with f(-X) does not hold (f(-X) is isomorphic to f)
    q, g = 5, 2
    curves = _random_curves(curvegen_mod, q, g, 20, seed=4242)
    neg = curves.astype(np.int64).copy()
    neg[:, 1::2] = (-neg[:, 1::2]) % q
    A = oracle_mod.count_curves(q, g, curves, kmax=1)
    B = oracle_mod.count_curves(q, g, neg.astype(np.int16), kmax=1)
    assert (A == B).all()
    assert not (A[:, 0] + B[:, 0] == 2 + q).all()


def _affine(row, q, a, b):
    """coefficients of f(aX + b) over F_q (q prime), constant term first"""
    d = len(row) - 1
    out = [0] * (d + 1)
    for i, c in enumerate(row):
        for j in range(i + 1):      # (aX+b)^i = sum_j C(i,j) a^j b^{i-j} X^j
            out[j] = (out[j] + c * math.comb(i, j) * pow(a, j, q) * pow(b, i - j, q)) % q
    return out


@pytest.mark.parametrize("q,g", [(5, 2), (7, 2), (13, 3)])
def test_gl2_invariance(oracle_mod, curvegen_mod, q, g):
    curves = _random_curves(curvegen_mod, q, g, 12, seed=555 + q)
    curves = curves[curves[:, 0] != 0]            # keeps the reversal in degree 2g+2
    base = oracle_mod.count_curves(q, g, curves, kmax=2)
    rng = np.random.default_rng(q)
    aff, scl, rev = [], [], []
    for row in curves:
        a, b, s = int(rng.integers(1, q)), int(rng.integers(0, q)), int(rng.integers(1, q))
        aff.append(_affine([int(v) for v in row], q, a, b))
        scl.append([(int(v) * s * s) % q for v in row])
        rev.append([int(v) for v in row[::-1]])
    for other in (aff, scl, rev):
        N = oracle_mod.count_curves(q, g, np.array(other, dtype=np.int16), kmax=2)
        assert (N == base).all()


@pytest.mark.parametrize("q,g,kmax", [(5, 2, 2), (9, 2, 2), (13, 3, 2), (3, 4, 3), (25, 2, 1)])
def test_model_and_root_independence(oracle_mod, curvegen_mod, q, g, kmax):
    curves = _random_curves(curvegen_mod, q, g, 10, seed=2024 + q)
    A = oracle_mod.count_curves(q, g, curves, kmax=kmax)
    B = oracle_mod.count_curves(q, g, curves, kmax=kmax, modulus_last=True)
    C = oracle_mod.count_curves(q, g, curves, kmax=kmax, root_last=True)
    assert (A == B).all() and (A == C).all()


def test_subfield_monotonicity(oracle_mod, curvegen_mod):
    # points over F_q are points over F_{q^2}: N_1 <= N_2, N_1 <= N_3, N_2 <= N_4
    q, g = 3, 3
    curves = _random_curves(curvegen_mod, q, g, 16, seed=8)
    N = oracle_mod.count_curves(q, g, curves, kmax=4)
    assert (N[:, 0] <= N[:, 1]).all() and (N[:, 0] <= N[:, 2]).all() and (N[:, 1] <= N[:, 3]).all()


def test_histogram_is_sorted_multiset(oracle_mod):
    rng = np.random.default_rng(3)
    N = rng.integers(0, 4, size=(500, 3)).astype(np.int32)
    keys, counts = oracle_mod.histogram(N)
    assert int(counts.sum()) == 500
    as_tuples = [tuple(r) for r in keys]
    assert as_tuples == sorted(set(as_tuples))
    for k, c in zip(as_tuples, counts):
        assert int(c) == int((N == np.array(k)).all(axis=1).sum())


def test_rejects_bad_input(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.count_curves(15, 2, np.zeros((1, 7), dtype=np.int16))
    with pytest.raises(ValueError):
        oracle_mod.count_curves(5, 2, np.array([[1, 0, 0, 0, 0, 0, 0]], dtype=np.int16))
    with pytest.raises(ValueError):
        oracle_mod.count_curves(5, 2, np.array([[5, 0, 0, 0, 0, 1, 0]], dtype=np.int16))


def test_table1_golden_is_the_oracle(oracle_mod):
    """tests/golden/table1_counts.txt holds oracle counts; recheck the small primes."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_counts.txt")
    rows = [list(map(int, l.split())) for l in open(path) if l.strip() and not l.startswith("#")]
    curve = [17, 12, 16, 11, 10, 13, 12]
    for p, n1, n2 in rows[:3]:
        r = np.array([[c % p for c in curve]], dtype=np.int16)
        assert oracle_mod.count_curves(p, 2, r, kmax=2)[0].tolist() == [n1, n2]
    for p, n1, n2 in rows:                                      # Weil bound, g = 2
        assert (n1 - p - 1) ** 2 <= 16 * p and (n2 - p * p - 1) ** 2 <= 16 * p * p
