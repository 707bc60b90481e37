"""The serving loop's logic on the CPU with a fake executor (no GPU): batch
packing and chunking, failure isolation, completion, histogram merging."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1805_11991_amd import serving


class FakeExecutor:
    """Completes a batch after `delay` polls; N[i] = row sum of codes, so the
    server's scatter-back can be checked exactly.  Fails any batch holding a
    request with q == 3 (to exercise failure isolation)."""

    def __init__(self, delay=1, fail_q=None):
        self.delay = delay
        self.fail_q = fail_q
        self.submitted = []

    def submit(self, jobs):
        if self.fail_q is not None and any(q == self.fail_q for q, _, _, _ in jobs):
            raise RuntimeError("simulated device failure")
        self.submitted.append([(q, g, len(c)) for q, g, c, _ in jobs])
        return {"jobs": jobs, "polls": 0}

    def poll(self, h):
        h["polls"] += 1
        return h["polls"] > self.delay

    def wait_any(self, hs):
        for h in hs:
            h["polls"] = self.delay + 1

    def collect(self, h):
        out = []
        for q, g, codes, want in h["jobs"]:
            N = np.repeat(codes.astype(np.int64).sum(axis=1, keepdims=True), g, axis=1).astype(np.int32)
            keys, cnt = np.unique(N, axis=0, return_counts=True)
            out.append((N, (keys.astype(np.int32), cnt.astype(np.uint64)) if want else None))
        return out


def _req(i, q, g, n, seed=0):
    rng = np.random.default_rng(seed + i)
    c = rng.integers(0, q, size=(n, 2 * g + 3)).astype(np.int16)
    c[:, -1] = np.maximum(c[:, -1], 1)
    return serving.Request(i, q, g, c)


def test_batches_respect_budget_and_split_large_requests():
    ex = FakeExecutor()
    srv = serving.Server(ex, batch_curves=1000, max_inflight=2)
    reqs = [_req(0, 13, 3, 2500), _req(1, 5, 2, 300), _req(2, 7, 4, 700), _req(3, 13, 3, 0)]
    for r in reqs:
        srv.submit(r)
    srv.drain()
    assert all(r.error is None for r in reqs)
    for batch in ex.submitted:
        assert sum(n for _, _, n in batch) <= 1000
    for r in reqs:
        expect = np.repeat(r.codes.astype(np.int64).sum(axis=1, keepdims=True), r.g, axis=1)
        assert np.array_equal(r.N, expect)
        keys, cnt = np.unique(expect, axis=0, return_counts=True)
        assert np.array_equal(r.hist[0], keys) and np.array_equal(r.hist[1], cnt.astype(np.uint64))
    assert reqs[0].latency is not None and srv.curves_done == 3500


def test_least_work_first_with_aging():
    # batches take the least work first; a chunk older than max_wait goes
    # ahead of newer ones whatever its size
    t = [0.0]
    ex = FakeExecutor(delay=0)
    srv = serving.Server(ex, batch_curves=920, max_inflight=1, clock=lambda: t[0], max_wait=1.0)
    big, s1, s2 = _req(0, 13, 4, 900), _req(1, 5, 2, 50), _req(2, 5, 2, 50)
    for r in (big, s1, s2):
        r.arrival = 0.0
        srv.submit(r)
    srv.step()
    assert ex.submitted == [[(5, 2, 50), (5, 2, 50)]]
    t[0] = 2.0
    s3 = _req(3, 5, 2, 50)
    s3.arrival = 2.0
    srv.submit(s3)
    srv.step()
    assert ex.submitted[1] == [(13, 4, 900)]
    srv.drain()
    assert ex.submitted[2] == [(5, 2, 50)]
    assert all(r.error is None and r.N is not None for r in (big, s1, s2, s3))


def test_invalid_requests_fail_alone():
    ex = FakeExecutor()
    srv = serving.Server(ex, batch_curves=1 << 12)
    good = _req(0, 13, 3, 100)
    bad = [serving.Request(1, 15, 2, np.ones((4, 7), np.int16)),            # not a prime power
           serving.Request(2, 13, 5, np.ones((4, 13), np.int16)),           # g out of range
           serving.Request(3, 13, 3, np.full((4, 9), 13, np.int16)),        # code out of range
           serving.Request(4, 13, 3, np.zeros((4, 9), np.int16)),           # degree
           serving.Request(5, 4099, 2, np.ones((4, 7), np.int16))]          # field too large
    for r in [good] + bad:
        srv.submit(r)
    srv.drain()
    assert good.error is None and good.N is not None
    assert all(r.error for r in bad)


def test_device_failure_isolated_to_its_request():
    ex = FakeExecutor(fail_q=3)
    srv = serving.Server(ex, batch_curves=1 << 12)
    a, b, c = _req(0, 13, 3, 50), _req(1, 3, 2, 50), _req(2, 5, 2, 50)
    for r in (a, b, c):
        srv.submit(r)
    srv.drain()
    assert a.error is None and c.error is None and b.error


def test_merge_hist():
    g = 2
    p1 = (np.array([[1, 2], [3, 4]], np.int32), np.array([2, 1], np.uint64))
    p2 = (np.array([[1, 2], [5, 6]], np.int32), np.array([3, 4], np.uint64))
    k, c = serving.merge_hist([p1, p2], g)
    assert k.tolist() == [[1, 2], [3, 4], [5, 6]] and c.tolist() == [5, 1, 4]


def test_poisson_shapes():
    shp = serving.poisson_requests(10.0, 500, 1)
    t = [s[0] for s in shp]
    assert all(b > a for a, b in zip(t, t[1:]))
    assert abs(np.mean(np.diff(t)) - 0.1) < 0.03
    for _, q, g, n, _ in shp:
        assert serving.odd_prime_power(q) and g in (2, 3, 4) and 1 <= n <= 1 << 20
        assert q < {2: 300, 3: 50, 4: 15}[g]
