"""The allocation-free entry point (hwc_count_curves_dev_noalloc) against
hwc_count_curves_dev: the same per-curve N_k and histogram, bit for bit, on
two calls in a row (the second with fewer rows, so it runs on what the first
left in the static scratch), on both counting paths and in the plain and
full-sweep forms; and the requests it must refuse before enqueueing anything.
"""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctxs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_11991_amd import hwcount
    z = hwcount.Context(device=0)
    m = hwcount.Context(device=0, mfma=True)
    yield {"zech": z, "mfma": m}
    z.close()
    m.close()


def _run(fn, q, g, d, n, hist=True):
    """fn runs on torch's current stream (a side stream), so reading the outputs waits for it."""
    import torch
    dev = d.device
    N = torch.full((n, g), -1, dtype=torch.int32, device=dev)
    if not hist:
        fn(q, g, d, N)
        return N.cpu().numpy(), None
    hk = torch.full((n, g), -1, dtype=torch.int32, device=dev)
    hc = torch.zeros(n, dtype=torch.int64, device=dev)
    hl = torch.zeros(1, dtype=torch.int64, device=dev)
    fn(q, g, d, N, hk, hc, hl)
    L = int(hl.item())
    return N.cpu().numpy(), (hk[:L].cpu().numpy(), hc[:L].cpu().numpy())


@pytest.mark.parametrize("path", ["zech", "mfma"])
@pytest.mark.parametrize("q,g,sizes,flags", [
    (13, 3, (200_003, 4_097), 0),
    (13, 4, (60_001, 1_031), 0),
    (13, 4, (20_011, 513), 2),      # HWC_PLAIN
    (5, 2, (100_000, 77), 1),       # HWC_FULL_SWEEP
    (9, 3, (50_021, 3_000), 0),     # prime power: Zech on both contexts
    (7, 2, (30_000, 1), 0),
])
def test_noalloc_matches_dev(ctxs, oracle_mod, curvegen_mod, path, q, g, sizes, flags):
    import torch
    ctx = ctxs[path]
    ctx.plan_info(q, g, flags)          # makes the plan resident
    big = curvegen_mod.sample(q, g, sizes[0], seed=curvegen_mod.BASE_SEED + 700 + q * 10 + g)
    for i, n in enumerate(sizes):
        rows = big[:n] if i == 0 else curvegen_mod.sample(q, g, n, seed=curvegen_mod.BASE_SEED + 800 + q + g)
        print(f"  noalloc {path} q={q} g={g} n={n} flags={flags} call {i + 1}", flush=True)
        # a stream of torch's own (not its default stream, whose handle is 0:
        # the library takes a null stream for its context stream)
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            d = torch.from_numpy(rows).to("cuda:0")
            Nd, Hd = _run(lambda *a: ctx.count_curves_dev(*a, flags=flags, stream=st), q, g, d, n)
            ctx.status(st)
            Na, Ha = _run(lambda *a: ctx.count_curves_dev_noalloc(*a, flags=flags, stream=st), q, g, d, n)
            ctx.status(st)
            assert np.array_equal(Na, Nd), (path, q, g, n, np.flatnonzero((Na != Nd).any(axis=1))[:5])
            assert np.array_equal(Ha[0], Hd[0]) and np.array_equal(Ha[1], Hd[1]), (path, q, g, n)
            # without the histogram too
            Nb, _ = _run(lambda *a: ctx.count_curves_dev_noalloc(*a, flags=flags, stream=st), q, g, d, n,
                         hist=False)
            ctx.status(st)
            assert np.array_equal(Nb, Nd)
        if i == 1:   # the smaller call against the oracle as well
            assert np.array_equal(Na, oracle_mod.count_curves(q, g, rows))


def test_noalloc_refuses_what_it_cannot_do(ctxs, curvegen_mod):
    import torch
    from paper_1805_11991_amd import hwcount
    with hwcount.Context(device=0, autotune_db=None) as fresh:
        rows = curvegen_mod.sample(11, 2, 100, seed=curvegen_mod.BASE_SEED + 900)
        d = torch.from_numpy(rows).to("cuda:0")
        N = torch.empty((100, 2), dtype=torch.int32, device="cuda:0")
        torch.cuda.synchronize()    # the calls below run on the context's own stream
        # the plan of (11, 2) was never built on this context: building allocates
        with pytest.raises(hwcount.HwcError) as ei:
            fresh.count_curves_dev_noalloc(11, 2, d, N)
        assert ei.value.code == hwcount.HWC_ERR_ARG
        fresh.plan_info(11, 2)
        fresh.count_curves_dev_noalloc(11, 2, d, N)
        fresh.status()          # waits for the context's stream
        assert np.array_equal(N.cpu().numpy(), fresh.count_curves(11, 2, rows)[0])
        # a request larger than the static scratch is refused before any launch
        n = 3 << 20
        big = torch.ones((n, 9), dtype=torch.int8, device="cuda:0")
        Nbig = torch.full((n, 3), -7, dtype=torch.int32, device="cuda:0")
        hk = torch.empty((n, 3), dtype=torch.int32, device="cuda:0")
        hc = torch.empty(n, dtype=torch.int64, device="cuda:0")
        hl = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        torch.cuda.synchronize()
        fresh.plan_info(13, 3)
        with pytest.raises(hwcount.HwcError) as ei:
            fresh.count_curves_dev_noalloc(13, 3, big, Nbig, hk, hc, hl)
        assert ei.value.code == hwcount.HWC_ERR_ARG
        assert "scratch" in str(ei.value)
        fresh.status()
        assert int((Nbig != -7).sum().item()) == 0
        with pytest.raises(hwcount.HwcError) as ei:
            fresh.count_curves_dev_noalloc(13, 3, big[:10], Nbig[:10], flags=hwcount.HWC_VALIDATE)
        assert ei.value.code == hwcount.HWC_ERR_ARG
