"""Serving on the GPU: every request's result in a mixed, chunked stream of
batches equals its result counted alone (also with a table-cache budget so
tight that plans are evicted mid-stream), the histograms equal the sorted
run-length histogram of N, a sample matches the oracle; batches on two
streams do not wait for each other; the table cache admits plans by its HBM
budget (HWC_ERR_OOM_BUDGET when one plan cannot fit, least recently used
eviction otherwise)."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_11991_amd import hwcount
    c = hwcount.Context(device=0)
    yield c
    c.close()


SHAPES = [(13, 3, 40000), (5, 2, 777), (3, 4, 5000), (13, 4, 20000), (191, 2, 30000), (9, 3, 3),
          (25, 2, 1), (11, 4, 12345), (41, 3, 9000), (13, 3, 64), (15, 2, 10), (7, 2, 100000)]


def _requests():
    from paper_1805_11991_amd import curvegen, serving
    reqs = []
    for i, (q, g, n) in enumerate(SHAPES):
        codes = curvegen.sample(q, g, n, seed=1000 + i) if q != 15 else np.ones((n, 2 * g + 3), np.int16)
        reqs.append(serving.Request(i, q, g, codes))
    return reqs


def _check_mix(ctx, reqs, oracle_mod, alone_ctx):
    for r in reqs:
        if r.q == 15:
            assert r.error and "prime power" in r.error
            continue
        assert r.error is None, r.error
        alone = alone_ctx.count_curves(r.q, r.g, r.codes)[0]
        assert np.array_equal(r.N, alone), (r.q, r.g, r.n)
        keys, cnt = np.unique(alone, axis=0, return_counts=True)
        assert np.array_equal(r.hist[0], keys) and np.array_equal(r.hist[1], cnt.astype(np.uint64))
        s = r.codes[: min(r.n, 200)]
        assert np.array_equal(r.N[: len(s)], oracle_mod.count_curves(r.q, r.g, s)), (r.q, r.g)


def test_mix_equals_alone(ctx, oracle_mod):
    from paper_1805_11991_amd import serving
    reqs = _requests()
    ex = serving.GpuExecutor(ctx, streams=2, batch_curves=1 << 15)
    srv = serving.Server(ex, batch_curves=1 << 15, max_inflight=2)
    for r in reqs:
        srv.submit(r)
    srv.drain()
    assert srv.batches > 4                     # several batches, large requests chunked
    _check_mix(ctx, reqs, oracle_mod, ctx)


def _plan_bytes(q, g):
    from paper_1805_11991_amd import hwcount
    with hwcount.Context(device=0, autotune_db=None) as c:
        c.plan_info(q, g)
        return c.stats()["table_bytes"]


def test_mix_equals_alone_under_tight_budget(ctx, oracle_mod):
    """A table-cache budget that holds only a few plans: the loop keeps
    serving, plans are evicted and rebuilt, and every result is unchanged."""
    from paper_1805_11991_amd import hwcount, serving
    big = max(_plan_bytes(q, g) for q, g, _ in SHAPES if q != 15)
    tight = hwcount.Context(device=0, hbm_budget_bytes=int(big * 1.5))
    try:
        reqs = _requests()
        ex = serving.GpuExecutor(tight, streams=2, batch_curves=1 << 14, max_jobs=4)
        srv = serving.Server(ex, batch_curves=1 << 14, max_inflight=2)
        for r in reqs:
            srv.submit(r)
        srv.drain()
        st = tight.stats()
        print(f"  tight budget {int(big * 1.5)} B: {st}", flush=True)
        assert st["evictions"] > 0
        assert st["table_bytes"] + st["pending_free_bytes"] <= int(big * 1.5)
        _check_mix(tight, reqs, oracle_mod, ctx)
    finally:
        tight.close()


def test_oom_budget_when_one_plan_cannot_fit(curvegen_mod):
    import torch
    from paper_1805_11991_amd import hwcount
    need = _plan_bytes(13, 4)
    c = hwcount.Context(device=0, hbm_budget_bytes=need // 2)
    try:
        d = torch.from_numpy(curvegen_mod.sample(13, 4, 100, seed=3)).cuda()
        N = torch.empty((100, 4), dtype=torch.int32, device="cuda")
        with pytest.raises(hwcount.HwcError) as ei:
            c.count_curves_dev(13, 4, d, N)
        assert ei.value.code == hwcount.HWC_ERR_OOM_BUDGET
        # a smaller plan still fits, and counts
        d5 = torch.from_numpy(curvegen_mod.sample(5, 2, 100, seed=4)).cuda()
        N5 = torch.empty((100, 2), dtype=torch.int32, device="cuda")
        c.count_curves_dev(5, 2, d5, N5)
        c.status()
    finally:
        c.close()


def test_lru_eviction_keeps_results(oracle_mod, curvegen_mod):
    """Budget for about two plans, three plans used in turn: each new plan
    evicts the least recently used one, and every count stays exact."""
    from paper_1805_11991_amd import hwcount
    fields = [(7, 3), (11, 3), (13, 3)]
    sizes = [_plan_bytes(q, g) for q, g in fields]
    budget = sizes[-1] + max(sizes[:-1]) + 4096
    c = hwcount.Context(device=0, hbm_budget_bytes=budget, autotune_db=None)
    try:
        for rep in range(2):
            for (q, g) in fields:
                rows = curvegen_mod.sample(q, g, 300, seed=q + rep)
                N, _ = c.count_curves(q, g, rows)
                assert np.array_equal(N, oracle_mod.count_curves(q, g, rows)), (q, g, rep)
                st = c.stats()
                assert st["table_bytes"] + st["pending_free_bytes"] <= budget
        st = c.stats()
        assert st["evictions"] >= 2 and st["plans_resident"] <= 2
    finally:
        c.close()


def test_batches_on_two_streams_do_not_wait_for_each_other(ctx, curvegen_mod):
    """Stream 1 is held by a spin kernel before its count; a count on stream 2
    issued afterwards completes while stream 1 is still held (the library no
    longer orders calls on different streams), and both results are exact."""
    import torch
    a = curvegen_mod.sample(13, 3, 4000, seed=501)
    b = curvegen_mod.sample(7, 4, 300, seed=502)
    ra, _ = ctx.count_curves(13, 3, a)
    rb, _ = ctx.count_curves(7, 4, b)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    Na = torch.empty((len(a), 3), dtype=torch.int32, device="cuda")
    Nb = torch.empty((len(b), 4), dtype=torch.int32, device="cuda")
    for s in (s1, s2):       # the streams' scratch, allocated before the timed part
        ctx.reserve(1 << 16, 4, stream=s)
    ctx.count_curves_dev(13, 3, da, Na, stream=s1)
    ctx.count_curves_dev(7, 4, db, Nb, stream=s2)
    torch.cuda.synchronize()
    # calibrate the spin kernel to a few hundred milliseconds
    cycles = 1 << 20
    while True:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(s1):
            e0.record()
            torch.cuda._sleep(cycles)
            e1.record()
        e1.synchronize()
        if e0.elapsed_time(e1) > 200 or cycles >= 1 << 32:
            break
        cycles *= 4
    with torch.cuda.stream(s1):
        torch.cuda._sleep(cycles)
    done1 = torch.cuda.Event()
    ctx.count_curves_dev(13, 3, da, Na, stream=s1)
    done1.record(s1)
    with torch.cuda.stream(s2):
        Nb.fill_(-1)
    ctx.count_curves_dev(7, 4, db, Nb, stream=s2)
    s2.synchronize()
    overlapped = not done1.query()
    torch.cuda.synchronize()
    ctx.status()
    assert overlapped, "the stream-2 count waited for stream 1"
    assert np.array_equal(Na.cpu().numpy(), ra)
    assert np.array_equal(Nb.cpu().numpy(), rb)
