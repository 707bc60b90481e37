"""GPU parity of the factorization partition lambda(f) (Sec. 1.1, eq. 1.2)
against the oracle's distinct-degree factorization, with the counts and the
(N, lambda) histogram, in every launch form."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_11991_amd import hwcount
    c = hwcount.Context(device=0)
    yield c
    c.close()


def _codes_from_oracle(mults):
    from paper_1805_11991_amd import hwcount
    return np.array([hwcount.lambda_code(m) for m in mults], dtype=np.uint32)


def _run(ctx, q, g, curves, flags=0, hist=True):
    import torch
    n = len(curves)
    d = torch.from_numpy(curves).cuda()
    N = torch.empty((n, g), dtype=torch.int32, device="cuda")
    lam = torch.empty(n, dtype=torch.int32, device="cuda")
    hk = torch.empty((max(n, 1), g + 1), dtype=torch.int32, device="cuda") if hist else None
    hc = torch.empty(max(n, 1), dtype=torch.int64, device="cuda") if hist else None
    hl = torch.zeros(1, dtype=torch.int64, device="cuda") if hist else None
    ctx.count_lambda_dev(q, g, d, N, lam, hk, hc, hl, flags=flags)
    ctx.status()
    out = (N.cpu().numpy(), lam.cpu().numpy().view(np.uint32))
    if hist:
        L = int(hl.item())
        out += (hk[:L].cpu().numpy(), hc[:L].cpu().numpy().astype(np.uint64))
    return out


CASES = [(3, 1, 300), (5, 1, 300), (3, 2, 800), (5, 2, 600), (7, 2, 400), (9, 2, 300), (13, 2, 300),
         (25, 2, 120), (3, 3, 400), (5, 3, 300), (13, 3, 300), (9, 3, 100), (17, 3, 60), (3, 4, 300),
         (5, 4, 150), (13, 4, 80), (37, 3, 40)]   # 37^3: the top level's sweep in tile parts


@pytest.mark.parametrize("q,g,n", CASES)
@pytest.mark.parametrize("flags", [0, 1, 2])       # orbit sweep, full sweep, plain form
def test_lambda_matches_oracle(lctx, oracle_mod, curvegen_mod, q, g, n, flags):
    curves = curvegen_mod.sample(q, g, n, seed=300 + q + 10 * g)
    N, lam, hk, hc = _run(lctx, q, g, curves, flags)
    assert np.array_equal(N, oracle_mod.count_curves(q, g, curves))
    want = _codes_from_oracle(oracle_mod.factor_degrees(q, g, curves))
    bad = np.flatnonzero(lam != want)
    assert bad.size == 0, (q, g, flags, bad[:5], lam[bad[:5]], want[bad[:5]], curves[bad[:5]])
    rows = np.concatenate([N.astype(np.int64), lam.astype(np.int64)[:, None]], axis=1)
    k, c = np.unique(rows, axis=0, return_counts=True)
    assert np.array_equal(hk.astype(np.int64), k)
    assert np.array_equal(hc, c.astype(np.uint64))


@pytest.mark.parametrize("q,g,n", [(13, 3, 5000), (5, 4, 2600), (3, 2, 4097), (7, 1, 1025)])
def test_lambda_several_tiles(lctx, oracle_mod, curvegen_mod, q, g, n):
    # the partition kernel works in passes of 1024 rows per workgroup and the
    # histogram in sort tiles of 4096 keys: several of each, ragged last ones
    curves = curvegen_mod.sample(q, g, n, seed=900 + q + 10 * g)
    N, lam, hk, hc = _run(lctx, q, g, curves)
    assert np.array_equal(N, oracle_mod.count_curves(q, g, curves))
    want = _codes_from_oracle(oracle_mod.factor_degrees(q, g, curves))
    assert np.array_equal(lam, want)
    rows = np.concatenate([N.astype(np.int64), lam.astype(np.int64)[:, None]], axis=1)
    k, c = np.unique(rows, axis=0, return_counts=True)
    assert np.array_equal(hk.astype(np.int64), k)
    assert np.array_equal(hc, c.astype(np.uint64))


def test_lambda_full_enumeration_g2_q5(lctx, oracle_mod, curvegen_mod):
    curves = curvegen_mod.enumerate_all(5, 2)
    N, lam, hk, hc = _run(lctx, 5, 2, curves)
    want = _codes_from_oracle(oracle_mod.factor_degrees(5, 2, curves))
    assert np.array_equal(lam, want)
    assert int(hc.sum()) == len(curves)


def test_lambda_full_size_g3_q13_sampled(lctx, oracle_mod, curvegen_mod):
    n = 1 << 24
    curves = curvegen_mod.sample(13, 3, n, seed=curvegen_mod.BASE_SEED + 1)
    N, lam = _run(lctx, 13, 3, curves, hist=False)
    assert not (lam == 0xFFFFFFFF).any()
    rng = np.random.default_rng(77)
    idx = np.unique(np.concatenate([rng.integers(0, n, 2000), [0, n - 1]]))
    want = _codes_from_oracle(oracle_mod.factor_degrees(13, 3, curves[idx]))
    assert np.array_equal(lam[idx], want)
    # every code decodes to a partition of 8
    from paper_1805_11991_amd import hwcount
    m = hwcount.lambda_multiplicities(np.unique(lam), 3)
    assert ((m * np.arange(1, 9)).sum(axis=1) == 8).all()


def test_lambda_needs_small_q(lctx, curvegen_mod):
    import torch
    from paper_1805_11991_amd import hwcount
    q = 10949                                           # prime, q - 1 > 10922
    c = torch.ones((4, 5), dtype=torch.int16, device="cuda")
    N = torch.empty((4, 1), dtype=torch.int32, device="cuda")
    lam = torch.empty(4, dtype=torch.int32, device="cuda")
    with pytest.raises(hwcount.HwcError):
        lctx.count_lambda_dev(q, 1, c, N, lam)
