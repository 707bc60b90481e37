"""Serving loop on the GPU: every request's result in a mixed, chunked stream
of batches equals its result counted alone, the histograms equal the sorted
run-length histogram of N, and a sample matches the oracle."""
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


def test_mix_equals_alone(ctx, oracle_mod):
    from paper_1805_11991_amd import curvegen, serving
    shapes = [(13, 3, 40000), (5, 2, 777), (3, 4, 5000), (13, 4, 20000), (191, 2, 30000), (9, 3, 3),
              (25, 2, 1), (11, 4, 12345), (41, 3, 9000), (13, 3, 64), (15, 2, 10), (7, 2, 100000)]
    reqs = []
    for i, (q, g, n) in enumerate(shapes):
        codes = curvegen.sample(q, g, n, seed=1000 + i) if q != 15 else np.ones((n, 2 * g + 3), np.int16)
        reqs.append(serving.Request(i, q, g, codes))
    srv = serving.Server(serving.GpuExecutor(ctx), batch_curves=1 << 15, max_inflight=2)
    for r in reqs:
        srv.submit(r)
    srv.drain()
    assert srv.batches > 4                     # several batches, large requests chunked
    for r in reqs:
        if r.q == 15:
            assert r.error and "prime power" in r.error
            continue
        assert r.error is None, r.error
        alone = ctx.count_curves(r.q, r.g, r.codes)[0]
        assert np.array_equal(r.N, alone), (r.q, r.g, r.n)
        keys, cnt = np.unique(alone, axis=0, return_counts=True)
        assert np.array_equal(r.hist[0], keys) and np.array_equal(r.hist[1], cnt.astype(np.uint64))
        s = r.codes[: min(r.n, 200)]
        assert np.array_equal(r.N[: len(s)], oracle_mod.count_curves(r.q, r.g, s)), (r.q, r.g)
