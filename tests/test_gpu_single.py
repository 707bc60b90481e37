"""One curve over large fields with the lane-per-x kernel (the single-curve
experiment of Table 1): N_1..N_k against the oracle, Table 1's curve over
F_{p^2} up to p = 3001, random curves of every genus, orbit and full sweeps."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# Table 1's curve, Y^2 = 12X^6 + 13X^5 + 10X^4 + 11X^3 + 16X^2 + 12X + 17, constant term first
TABLE1 = [17, 12, 16, 11, 10, 13, 12]


@pytest.fixture(scope="module")
def sctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_11991_amd import hwcount
    c = hwcount.Context(device=0)
    yield c
    c.close()


def _table1():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_counts.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    return [(int(a), int(b), int(c)) for a, b, c in rows]


@pytest.mark.parametrize("p,N1,N2", _table1())
def test_table1_curve(sctx, p, N1, N2):
    """All primes of Table 1 against the oracle's counts (tests/golden)."""
    row = np.array([c % p for c in TABLE1], dtype=np.int16)
    N, t = sctx.count_single(p, 2, row, 2)
    assert N.tolist() == [N1, N2], p
    assert t["kernel_ms"] > 0
    N, _ = sctx.count_single(p, 2, row, 2, flags=1)   # full sweep
    assert N.tolist() == [N1, N2], p


@pytest.mark.parametrize("q,g,kmax", [(3, 1, 8), (5, 2, 6), (7, 3, 5), (9, 2, 4), (13, 4, 4), (25, 3, 3),
                                      (27, 2, 3), (101, 1, 3), (3, 4, 10)])
@pytest.mark.parametrize("flags", [0, 1])
def test_random_curves(sctx, oracle_mod, curvegen_mod, q, g, kmax, flags):
    rows = curvegen_mod.sample(q, g, 4, seed=q * 10 + g, dtype=np.int16)
    ref = oracle_mod.count_curves(q, g, rows, kmax=kmax)
    for r, want in zip(rows, ref):
        N, _ = sctx.count_single(q, g, r, kmax, flags=flags)
        assert np.array_equal(N, want.astype(np.int64)), (q, g, kmax, flags, r, N, want)


def test_single_agrees_with_batched(sctx, curvegen_mod):
    rows = curvegen_mod.sample(13, 3, 16, seed=5)
    N, _ = sctx.count_curves(13, 3, rows)
    for r, want in zip(rows, N):
        got, _ = sctx.count_single(13, 3, r, 3)
        assert np.array_equal(got, want.astype(np.int64))
