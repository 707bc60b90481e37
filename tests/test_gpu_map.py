"""The map N_{g,q} of eq. (1.2) by Algorithm 1 (reduced representatives,
multiplicities, twist doubling) equals the same map taken over the full
enumeration of square-free polynomials: from the oracle's counts and
factorizations for small fields, from the device's own full-enumeration
counts (themselves oracle-checked elsewhere) for larger ones."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_11991_amd import hwcount
    c = hwcount.Context(device=0)
    yield c
    c.close()


def _map_from_rows(q, g, N, codes):
    a = np.array([q ** k + 1 for k in range(1, g + 1)], dtype=np.int64) - N.astype(np.int64)
    rows = np.concatenate([a, codes.astype(np.int64)[:, None]], axis=1)
    k, c = np.unique(rows, axis=0, return_counts=True)
    return k, c.astype(np.uint64)


def _total(q, g):
    return (q - 1) * (q ** (2 * g + 2) - q ** (2 * g + 1)) + (q - 1) * (q ** (2 * g + 1) - q ** (2 * g))


def _check(mctx, q, g, ref_keys, ref_counts):
    keys, counts, reps = mctx.count_map(q, g)
    assert int(counts.sum()) == _total(q, g)
    assert np.array_equal(keys.astype(np.int64), ref_keys), (q, g, len(keys), len(ref_keys))
    assert np.array_equal(counts, ref_counts), (q, g)
    return reps


@pytest.mark.parametrize("q,g", [(3, 1), (5, 1), (7, 1), (9, 1), (11, 1), (3, 2), (5, 2), (7, 2), (9, 2), (3, 3),
                                 (3, 4)])
def test_map_equals_oracle_full_enumeration(mctx, oracle_mod, curvegen_mod, q, g):
    from paper_1805_11991_amd import hwcount
    rows = curvegen_mod.enumerate_all(q, g)
    assert len(rows) == _total(q, g)
    N = oracle_mod.count_curves(q, g, rows)
    codes = np.array([hwcount.lambda_code(m) for m in oracle_mod.factor_degrees(q, g, rows)], dtype=np.int64)
    k, c = _map_from_rows(q, g, N, codes)
    reps = _check(mctx, q, g, k, c)
    assert reps < len(rows)


@pytest.mark.parametrize("q,g", [(5, 3), (11, 2), (7, 3)])
def test_map_equals_device_full_enumeration(mctx, curvegen_mod, q, g):
    """The full enumeration counted on the device with its (N, lambda)
    histogram, turned into (a, lambda) keys."""
    import torch
    rows = curvegen_mod.enumerate_all(q, g)
    n = len(rows)
    d = torch.from_numpy(rows).cuda()
    N = torch.empty((n, g), dtype=torch.int32, device="cuda")
    lam = torch.empty(n, dtype=torch.int32, device="cuda")
    hk = torch.empty((n, g + 1), dtype=torch.int32, device="cuda")
    hc = torch.empty(n, dtype=torch.int64, device="cuda")
    hl = torch.zeros(1, dtype=torch.int64, device="cuda")
    mctx.count_lambda_dev(q, g, d, N, lam, hk, hc, hl)
    mctx.status()
    L = int(hl.item())
    keys = hk[:L].cpu().numpy().astype(np.int64)
    cnt = hc[:L].cpu().numpy().astype(np.uint64)
    del d, N, lam, hk, hc
    keys[:, :g] = np.array([q ** k + 1 for k in range(1, g + 1)], dtype=np.int64) - keys[:, :g]
    order = np.lexsort(keys.T[::-1])
    _check(mctx, q, g, keys[order], cnt[order])
