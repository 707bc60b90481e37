"""Small finite fields by explicit tables, for brute-force pins of the oracle.

These models are deliberately different from the oracle's: extensions are
built as B[s]/(h(s)) with h the first monic irreducible polynomial over the
base B found by root search (degree 2 or 3 only), not as F_p[t] modulo a
primitive polynomial.  Point counts are taken by counting pairs (x, y) with
y^2 = f(x), without any quadratic character.
"""
from __future__ import annotations

import itertools

import numpy as np


class TableField:
    """A field of size Q given by add/mul tables over element ids 0..Q-1
    (0 is zero, 1 is one)."""

    def __init__(self, add: np.ndarray, mul: np.ndarray):
        self.add = add
        self.mul = mul
        self.Q = add.shape[0]
        self.neg = np.argmin(add, axis=1)  # b with a + b = 0

    @staticmethod
    def prime(p: int) -> "TableField":
        r = np.arange(p)
        return TableField((r[:, None] + r[None, :]) % p, (r[:, None] * r[None, :]) % p)

    def extend(self, degree: int) -> tuple["TableField", list]:
        """B[s]/(h) with h the first monic irreducible of the given degree
        (2 or 3: irreducible iff no root in B).  Returns the field and h.
        Element id of (b_0, .., b_{m-1}) is sum_i b_i * Q^i, so base elements
        keep their ids."""
        assert degree in (2, 3)
        B = self.Q
        h = None
        for coeffs in itertools.product(range(B), repeat=degree):
            # h(s) = s^m + coeffs[m-1] s^{m-1} + ... + coeffs[0]
            ok = True
            for r in range(B):
                v = 1
                for c in reversed(coeffs):
                    v = self.add[self.mul[v, r], c]
                # v = r^m + ... evaluated by Horner with leading 1
                if v == 0:
                    ok = False
                    break
            if ok:
                h = list(coeffs)
                break
        assert h is not None
        m = degree
        Q = B ** m
        digits = np.array([[(e // B ** i) % B for i in range(m)] for e in range(Q)])
        ids = lambda d: int(sum(int(d[i]) * B ** i for i in range(m)))
        add = np.zeros((Q, Q), dtype=np.int64)
        mul = np.zeros((Q, Q), dtype=np.int64)
        negh = [self.neg[c] for c in h]
        for a in range(Q):
            da = digits[a]
            for b in range(a, Q):
                db = digits[b]
                s = [self.add[da[i], db[i]] for i in range(m)]
                add[a, b] = add[b, a] = ids(s)
                prod = [0] * (2 * m - 1)
                for i in range(m):
                    for j in range(m):
                        prod[i + j] = self.add[prod[i + j], self.mul[da[i], db[j]]]
                for d in range(2 * m - 2, m - 1, -1):
                    top = prod[d]
                    prod[d] = 0
                    for i in range(m):
                        prod[d - m + i] = self.add[prod[d - m + i], self.mul[top, negh[i]]]
                mul[a, b] = mul[b, a] = ids(prod[:m])
        return TableField(add, mul), h

    def count_points(self, coeffs: list[int], g: int) -> int:
        """#{(x, y) in E^2 : y^2 = f(x)} + #{y : y^2 = c_{2g+2}} (points at
        infinity of the model in P(1, g+1, 1)).  coeffs are element ids,
        constant term first, length 2g+3."""
        Q = self.Q
        xs = np.arange(Q)
        sq = self.mul[xs, xs]
        nroots = np.bincount(sq, minlength=Q)   # #{y : y^2 = v}
        y = np.full(Q, coeffs[-1], dtype=np.int64)
        for c in reversed(coeffs[:-1]):
            y = self.add[self.mul[y, xs], c]
        return int(nroots[y].sum() + nroots[coeffs[-1]])


def prime_power_model(p: int, e: int, P: list[int]) -> TableField:
    """F_{p^e} = F_p[t]/(P) with explicit tables, element id = sum_i d_i p^i
    for sum_i d_i t^i (the coefficient-code convention).  P is given
    constant term first with leading 1."""
    Q = p ** e
    dig = [[(v // p ** i) % p for i in range(e)] for v in range(Q)]
    add = np.zeros((Q, Q), dtype=np.int64)
    mul = np.zeros((Q, Q), dtype=np.int64)
    for a in range(Q):
        for b in range(Q):
            s = [(dig[a][i] + dig[b][i]) % p for i in range(e)]
            add[a, b] = sum(s[i] * p ** i for i in range(e))
            prod = [0] * (2 * e - 1)
            for i in range(e):
                for j in range(e):
                    prod[i + j] += dig[a][i] * dig[b][j]
            for d in range(2 * e - 2, e - 1, -1):
                top = prod[d] % p
                prod[d] = 0
                for i in range(e):
                    prod[d - e + i] -= top * P[i]
            mul[a, b] = sum((prod[i] % p) * p ** i for i in range(e))
    return TableField(add, mul)
