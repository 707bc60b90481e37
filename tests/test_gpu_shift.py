"""Dense translates on the GPU: rows with zero coefficients are counted as
f(x + t) (same N_k, factorization pattern and discriminant, see
test_translation_pins.py).  Parity with the oracle on the caller's rows,
identical results with translation switched off, the caller's buffer left
as it was, and the multi-plan batch path."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_11991_amd import hwcount
    c = hwcount.Context(device=0)
    yield c
    c.close()


def _sparse_rows(curvegen_mod, q, g, n, seed, frac=0.35):
    rows = curvegen_mod.sample(q, g, n, seed=seed)
    rng = np.random.default_rng(seed)
    low = rng.random((n, rows.shape[1] - 2)) < frac
    rows[:, :-2][low] = 0
    return rows


def _count(ctx, q, g, rows, shift, flags=0):
    import torch
    from paper_1805_11991_amd import hwcount as hw
    # translates serve the Zech-logarithm path; the matrix-core path needs none
    ctx.set_plan_option(q, g, hw.HWC_OPT_MFMA, 0, flags & hw.HWC_FULL_SWEEP)
    ctx.set_plan_option(q, g, hw.HWC_OPT_SHIFT, shift, flags & hw.HWC_FULL_SWEEP)
    n = len(rows)
    d = torch.from_numpy(rows).cuda()
    before = d.clone()
    N = torch.empty((n, g), dtype=torch.int32, device="cuda")
    hk = torch.empty((n, g), dtype=torch.int32, device="cuda")
    hc = torch.empty(n, dtype=torch.int64, device="cuda")
    hl = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.count_curves_dev(q, g, d, N, hk, hc, hl, flags=flags)
    # the partition codes too (rows that are not square-free get the invalid code)
    N2 = torch.empty((n, g), dtype=torch.int32, device="cuda")
    lam = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.count_lambda_dev(q, g, d, N2, lam, flags=flags)
    ctx.status()
    assert torch.equal(d, before), "the caller's rows were modified"
    assert torch.equal(N, N2)
    L = int(hl.item())
    return N.cpu().numpy(), lam.cpu().numpy(), hk[:L].cpu().numpy(), hc[:L].cpu().numpy()


@pytest.mark.parametrize("q,g", [(3, 2), (3, 4), (5, 3), (9, 3), (13, 3), (13, 4), (25, 2), (27, 2), (31, 3)])
@pytest.mark.parametrize("flags", [0, 1, 2])   # batched orbit, full sweep, plain
def test_translated_rows_match_oracle(sctx, oracle_mod, curvegen_mod, q, g, flags):
    n = 4000 if g < 4 else 1500
    rows = _sparse_rows(curvegen_mod, q, g, n, seed=77 * q + g)
    on = _count(sctx, q, g, rows, 1, flags)
    off = _count(sctx, q, g, rows, 0, flags)
    for a, b in zip(on, off):
        assert np.array_equal(a, b)
    assert np.array_equal(on[0], oracle_mod.count_curves(q, g, rows))


def test_rows_without_dense_translate_keep_their_form(sctx, oracle_mod, curvegen_mod):
    # over F_3 most sparse rows of degree 8 have no dense translate among t = 1, 2
    rows = _sparse_rows(curvegen_mod, 3, 3, 3000, seed=5, frac=0.6)
    on = _count(sctx, 3, 3, rows, 1)
    assert np.array_equal(on[0], oracle_mod.count_curves(3, 3, rows))


def test_batch_jobs_with_and_without_translates(sctx, oracle_mod, curvegen_mod):
    import torch
    specs = [(13, 3, 3000), (37, 2, 2000), (9, 4, 1200), (5, 2, 2500)]   # q = 37 has no step table
    jobs, want = [], []
    for i, (q, g, n) in enumerate(specs):
        rows = _sparse_rows(curvegen_mod, q, g, n, seed=300 + i)
        want.append(oracle_mod.count_curves(q, g, rows))
        jobs.append(dict(q=q, g=g, coeffs=torch.from_numpy(rows).cuda(),
                         out=torch.empty((n, g), dtype=torch.int32, device="cuda")))
    sctx.count_batch([dict(q=j["q"], g=j["g"], d_coeffs=j["coeffs"], d_out_N=j["out"]) for j in jobs])
    sctx.status()
    for j, w in zip(jobs, want):
        assert np.array_equal(j["out"].cpu().numpy(), w), (j["q"], j["g"])


def test_translate_entry_point(sctx, oracle_mod, curvegen_mod):
    import torch
    from paper_1805_11991_amd import hwcount as hw
    q, g = 13, 3
    rows = _sparse_rows(curvegen_mod, q, g, 5000, seed=11)
    d = torch.from_numpy(rows).cuda()
    out = torch.empty_like(d)
    sctx.set_plan_option(q, g, hw.HWC_OPT_SHIFT, 1)
    sctx.translate_dev(q, g, d, out)
    sctx.status()
    t = out.cpu().numpy().astype(np.int64)
    r = rows.astype(np.int64)
    # same leading coefficient and degree; rows that were dense are unchanged
    assert np.array_equal(t[:, -1], r[:, -1])
    deg = np.where(r[:, -1] != 0, r.shape[1] - 1, r.shape[1] - 2)
    below = np.arange(r.shape[1])[None, :] < deg[:, None]
    dense_in = ((r != 0) | ~below).all(axis=1)
    assert np.array_equal(t[dense_in], r[dense_in])
    # most sparse rows found a dense translate, and every output row counts as the input row
    dense_out = ((t != 0) | ~below).all(axis=1)
    assert dense_out[~dense_in].mean() > 0.9
    assert np.array_equal(oracle_mod.count_curves(q, g, t), oracle_mod.count_curves(q, g, rows))
    # above q = 32 rows are copied
    rows37 = _sparse_rows(curvegen_mod, 37, 2, 2000, seed=12)
    d37 = torch.from_numpy(rows37).cuda()
    o37 = torch.empty_like(d37)
    sctx.translate_dev(37, 2, d37, o37)
    sctx.status()
    assert np.array_equal(o37.cpu().numpy(), rows37)
    with pytest.raises(hw.HwcError):
        sctx.translate_dev(q, g, d, d)


@pytest.mark.parametrize("q,p,e,g", [(13, 13, 1, 3), (31, 31, 1, 4), (5, 5, 1, 2), (7, 7, 1, 1),
                                     (9, 3, 2, 3), (27, 3, 3, 2)])
def test_translate_takes_the_first_dense_t(sctx, oracle_mod, curvegen_mod, q, p, e, g):
    """Each row with a zero below its leading coefficient becomes f(x + t) for
    the first t = 1 .. min(q - 1, 8) that leaves none (prime q: the integer
    matrix form of the translate; prime powers: the step table), computed
    here by the binomial theorem over F_q from the oracle's field product."""
    import torch
    from paper_1805_11991_amd import hwcount as hw
    from test_translation_pins import _translate
    n = 160
    rows = _sparse_rows(curvegen_mod, q, g, n, seed=900 + q * 5 + g, frac=0.3)
    nc = rows.shape[1]
    want = rows.astype(np.int64).copy()
    for r in range(n):
        row = [int(v) for v in rows[r]]
        d = nc - 1 if row[-1] else nc - 2
        if all(row[i] != 0 for i in range(d)):
            continue
        for t in range(1, min(q - 1, 8) + 1):
            v = _translate(oracle_mod, row, t, p, e)
            if all(v[i] != 0 for i in range(d)):
                want[r] = v
                break
    sctx.set_plan_option(q, g, hw.HWC_OPT_SHIFT, 1)
    d = torch.from_numpy(rows).cuda()
    out = torch.empty_like(d)
    sctx.translate_dev(q, g, d, out)
    sctx.status()
    assert np.array_equal(out.cpu().numpy().astype(np.int64), want)
