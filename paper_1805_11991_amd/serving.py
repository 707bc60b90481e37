"""Serving loop: continuous batching of curve-count requests of mixed (q, g).

Requests arrive over time.  Pending requests are admitted into the next batch
while the batch has room: at most `batch_curves` curves and, when the executor
states one, at most its per-batch device bytes (codes, N and histogram
buffers); a request larger than that is split into chunks that ride in
successive batches.  A batch launches as soon as one of the executor's slots
(a stream with its own preallocated device arena and library scratch) is
free, so batches in flight overlap on the device: the uploads, kernels and
downloads of one run beside another's.  Each batch is one call of the
library's multi-plan persistent launch (``hwc_count_batch``).  Field tables
stay resident in the context's device cache, which admits plans against its
HBM budget (least recently used plans are evicted; their memory is freed once
the work reading it is done).  A finished batch is detected by an event;
results are scattered back to their requests and a request completes when its
last chunk does.

A request that cannot be served (bad q or g, bad coefficients, a field too
large, tables over the HBM budget) fails on its own; the loop keeps serving
the others.  Per-request latency is completion minus arrival time.

The executor is an interface: ``GpuExecutor`` runs batches on the GPU through
the C ABI; tests drive the same loop with a fake executor on the CPU.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque

import numpy as np


def odd_prime_power(q: int) -> bool:
    if q < 3 or q % 2 == 0:
        return False
    p = next((d for d in range(3, int(math.isqrt(q)) + 1, 2) if q % d == 0), q)
    while q % p == 0:
        q //= p
    return q == 1


MAX_FIELD = 1 << 24


@dataclasses.dataclass
class Request:
    rid: int
    q: int
    g: int
    codes: np.ndarray                  # [n, 2g+3] int8/int16, constant term first
    arrival: float = 0.0
    want_hist: bool = True
    # filled by the server
    N: np.ndarray | None = None
    hist: tuple[np.ndarray, np.ndarray] | None = None
    error: str | None = None
    done_at: float | None = None
    chunks_left: int = 0
    _parts: list = dataclasses.field(default_factory=list)

    @property
    def n(self) -> int:
        return int(self.codes.shape[0])

    @property
    def latency(self) -> float | None:
        return None if self.done_at is None else self.done_at - self.arrival


@dataclasses.dataclass
class Chunk:
    req: Request
    lo: int
    hi: int
    seq: int = 0                       # order of intake


def work_estimate(q: int, g: int, n: int) -> float:
    """Relative device work of n curves of genus g over F_q: the top level's
    points swept with the Frobenius orbits, q^g / g per curve, dominates."""
    return n * (q ** g) / g


def validate(req: Request) -> str | None:
    """Host-side checks, so a bad request never reaches a batch."""
    if not odd_prime_power(req.q):
        return f"q={req.q} is not an odd prime power"
    if not 1 <= req.g <= 4:
        return f"g={req.g} outside 1..4"
    if req.q ** req.g > MAX_FIELD:
        return f"F_{{q^g}} larger than {MAX_FIELD} elements"
    c = req.codes
    if c.ndim != 2 or c.shape[1] != 2 * req.g + 3:
        return f"coefficients must be [n, {2 * req.g + 3}]"
    if c.dtype == np.int8 and req.q > 127:
        return "int8 codes need q <= 127"
    if c.size and (int(c.min()) < 0 or int(c.max()) >= req.q):
        return "coefficient code out of range"
    if c.size and np.any((c[:, -1] == 0) & (c[:, -2] == 0)):
        return "degree below 2g+1"
    return None


def merge_hist(parts: list[tuple[np.ndarray, np.ndarray]], g: int):
    """Merge sorted (tuples, counts) histograms of the chunks of one request."""
    parts = [p for p in parts if len(p[0])]
    if not parts:
        return np.zeros((0, g), np.int32), np.zeros(0, np.uint64)
    if len(parts) == 1:
        return parts[0]
    keys = np.concatenate([p[0] for p in parts])
    counts = np.concatenate([p[1] for p in parts])
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    tot = np.zeros(len(uniq), np.uint64)
    np.add.at(tot, inv.reshape(-1), counts)
    return uniq.astype(np.int32), tot


class Server:
    def __init__(self, executor, batch_curves: int = 1 << 22, max_inflight: int = 2, clock=time.perf_counter,
                 max_jobs: int | None = None, max_wait: float = 0.05):
        self.ex = executor
        # batches take the least work first, so that small requests do not
        # wait behind large ones; a chunk that has waited max_wait seconds
        # (from its request's arrival) goes ahead of the rest, oldest first
        self.max_wait = max_wait
        self._seq = 0
        self.batch_curves = batch_curves
        # an executor with slots of its own bounds the batches in flight and their bytes
        self.max_inflight = min(max_inflight, getattr(executor, "slots", max_inflight))
        self.batch_bytes = getattr(executor, "batch_bytes", None)
        self.max_jobs = max_jobs or getattr(executor, "max_jobs", 1 << 16)
        self.clock = clock
        self.pending: deque[Chunk] = deque()
        self.inflight: deque = deque()      # (handle, [chunks])
        self.completed: list[Request] = []
        self.curves_done = 0
        self.batches = 0

    # -- intake
    def submit(self, req: Request):
        err = validate(req)
        if err:
            self._finish(req, error=err)
            return
        n = req.n
        if n == 0:
            req.N = np.zeros((0, req.g), np.int32)
            req.hist = (np.zeros((0, req.g), np.int32), np.zeros(0, np.uint64))
            self._finish(req)
            return
        per = self.batch_curves
        if self.batch_bytes is not None:   # a chunk must fit one batch's device bytes
            per_curve = -(-self.ex.job_bytes(req.q, req.g, 1024, req.codes.dtype, req.want_hist) // 1024)
            per = max(1, min(per, (self.batch_bytes - 4096) // per_curve))
        req.chunks_left = math.ceil(n / per)
        for lo in range(0, n, per):
            self.pending.append(Chunk(req, lo, min(n, lo + per), self._seq))
            self._seq += 1

    # -- the loop
    def step(self) -> int:
        """Collects finished batches and launches new ones; returns the number
        of requests completed in this step."""
        done_before = len(self.completed)
        while self.inflight and self.ex.poll(self.inflight[0][0]):
            handle, chunks = self.inflight.popleft()
            self._collect(handle, chunks)
        while self.pending and len(self.inflight) < self.max_inflight:
            batch, room, room_b = [], self.batch_curves, self.batch_bytes
            taken = set()
            for ch in self._order(self.clock()):
                if len(batch) >= self.max_jobs:
                    break
                m = ch.hi - ch.lo
                b = self._bytes(ch)
                if m > room or (room_b is not None and b > room_b):
                    continue                  # a smaller chunk may still fit
                taken.add(ch.seq)
                if ch.req.error:          # an earlier chunk of the request failed
                    continue
                batch.append(ch)
                room -= m
                if room_b is not None:
                    room_b -= b
            self.pending = deque(ch for ch in self.pending if ch.seq not in taken)
            if not batch:
                break
            self._launch(batch)
        return len(self.completed) - done_before

    def drain(self):
        while self.pending or self.inflight:
            if not self.step():
                self.ex.wait_any([h for h, _ in self.inflight])

    # -- internals
    def _order(self, now: float) -> list[Chunk]:
        def key(ch: Chunk):
            if now - ch.req.arrival >= self.max_wait:
                return (0, 0.0, ch.seq)
            return (1, work_estimate(ch.req.q, ch.req.g, ch.hi - ch.lo), ch.seq)
        return sorted(self.pending, key=key)

    def _bytes(self, ch: Chunk) -> int:
        if self.batch_bytes is None:
            return 0
        return self.ex.job_bytes(ch.req.q, ch.req.g, ch.hi - ch.lo, ch.req.codes.dtype, ch.req.want_hist)

    def _launch(self, batch: list[Chunk]):
        try:
            handle = self.ex.submit([(c.req.q, c.req.g, c.req.codes[c.lo:c.hi], c.req.want_hist) for c in batch])
            self.inflight.append((handle, batch))
            self.batches += 1
        except Exception:
            # isolate the failing request(s): run each chunk on its own
            for c in batch:
                free = getattr(self.ex, "free_slots", None)
                while free is not None and free() == 0 and self.inflight:
                    self._collect(*self.inflight.popleft())    # wait for a slot
                try:
                    handle = self.ex.submit([(c.req.q, c.req.g, c.req.codes[c.lo:c.hi], c.req.want_hist)])
                    self.inflight.append((handle, [c]))
                    self.batches += 1
                except Exception as e:
                    self._fail_chunk(c, str(e))

    def _collect(self, handle, chunks: list[Chunk]):
        try:
            results = self.ex.collect(handle)
        except Exception as e:
            for c in chunks:
                self._fail_chunk(c, str(e))
            return
        for c, (N, hist) in zip(chunks, results):
            req = c.req
            if req.error:
                continue
            req._parts.append((c.lo, N, hist))
            self.curves_done += c.hi - c.lo
            req.chunks_left -= 1
            if req.chunks_left == 0:
                req._parts.sort(key=lambda t: t[0])
                req.N = np.concatenate([p[1] for p in req._parts]) if len(req._parts) > 1 else req._parts[0][1]
                if req.want_hist:
                    req.hist = merge_hist([p[2] for p in req._parts], req.g)
                req._parts = []
                self._finish(req)

    def _fail_chunk(self, c: Chunk, msg: str):
        if not c.req.error:
            self._finish(c.req, error=msg)

    def _finish(self, req: Request, error: str | None = None):
        req.error = error
        req.done_at = self.clock()
        self.completed.append(req)


class GpuExecutor:
    """Runs batches with hwc_count_batch, one batch per slot.  A slot is a
    stream with its own device arena (codes, N and histogram buffers of up
    to `batch_bytes`), pinned host staging for the uploads and downloads,
    and library scratch preallocated with hwc_ctx_reserve; nothing is
    allocated per batch, and batches on different slots overlap."""

    ALIGN = 256

    def __init__(self, ctx, streams: int = 2, batch_curves: int = 1 << 22, max_jobs: int = 256):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.max_jobs = max_jobs
        # worst case per curve: int16 codes at g = 4, N, histogram keys and counts
        self.batch_bytes = batch_curves * self.job_bytes(13, 4, 1, np.int16, True) + max_jobs * 4 * self.ALIGN
        self.slots = streams
        self._free = list(range(streams))
        self._s = []
        for _ in range(streams):
            st = torch.cuda.Stream()
            ctx.reserve(batch_curves, max_jobs, stream=st)
            self._s.append({"stream": st,
                            "dev": torch.empty(self.batch_bytes, dtype=torch.uint8, device="cuda"),
                            "h_in": torch.empty(self.batch_bytes, dtype=torch.uint8).pin_memory(),
                            "h_out": torch.empty(self.batch_bytes, dtype=torch.uint8).pin_memory(),
                            "d_len": torch.zeros(max_jobs, dtype=torch.int64, device="cuda"),
                            "h_len": torch.zeros(max_jobs, dtype=torch.int64).pin_memory()})

    @classmethod
    def _al(cls, b: int) -> int:
        return (b + cls.ALIGN - 1) // cls.ALIGN * cls.ALIGN

    @classmethod
    def job_bytes(cls, q, g, n, dtype, want_hist) -> int:
        cb = np.dtype(dtype).itemsize
        b = cls._al(n * (2 * g + 3) * cb) + cls._al(n * g * 4)
        if want_hist:
            b += cls._al(max(n, 1) * g * 4) + cls._al(max(n, 1) * 8)
        return b

    def free_slots(self) -> int:
        return len(self._free)

    def submit(self, jobs):
        torch = self.torch
        if not self._free:
            raise RuntimeError("no free slot")
        if len(jobs) > self.max_jobs:
            raise RuntimeError("too many jobs for one batch")
        k = self._free.pop(0)
        sl = self._s[k]
        s = sl["stream"]
        dev, h_in, h_out = sl["dev"], sl["h_in"], sl["h_out"]
        hv_in = h_in.numpy()
        off = 0

        def take(nbytes):
            nonlocal off
            if off + nbytes > self.batch_bytes:
                raise RuntimeError("batch larger than the slot's arena")
            o = off
            off += self._al(nbytes)
            return o

        try:
            bufs, views = [], []
            with torch.cuda.stream(s):
                for i, (q, g, codes, want_hist) in enumerate(jobs):
                    n = codes.shape[0]
                    c = np.ascontiguousarray(codes)
                    o = take(c.nbytes)
                    hv_in[o:o + c.nbytes] = c.view(np.uint8).reshape(-1)
                    d = dev[o:o + c.nbytes]
                    d.copy_(h_in[o:o + c.nbytes], non_blocking=True)
                    tdt = torch.int8 if c.dtype == np.int8 else torch.int16
                    b = {"q": q, "g": g, "d_coeffs": d.view(tdt).view(n, 2 * g + 3)}
                    on = take(n * g * 4)
                    b["d_out_N"] = dev[on:on + n * g * 4].view(torch.int32).view(n, g)
                    view = {"N": (on, n, g)}
                    if want_hist:
                        m = max(n, 1)
                        ok, oc = take(m * g * 4), take(m * 8)
                        b["d_hist_keys"] = dev[ok:ok + m * g * 4].view(torch.int32).view(m, g)
                        b["d_hist_counts"] = dev[oc:oc + m * 8].view(torch.int64)
                        b["d_hist_len"] = sl["d_len"][i:i + 1]
                        view["hist"] = (ok, oc, g)
                    bufs.append(b)
                    views.append(view)
            from .hwcount import HWC_NO_GRAPH
            self.ctx.count_batch(bufs, flags=HWC_NO_GRAPH, stream=s)
            with torch.cuda.stream(s):
                for i, v in enumerate(views):
                    on, n, g = v["N"]
                    h_out[on:on + n * g * 4].copy_(dev[on:on + n * g * 4], non_blocking=True)
                    if "hist" in v:
                        sl["h_len"][i:i + 1].copy_(sl["d_len"][i:i + 1], non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(s)
        except Exception:
            self._free.insert(0, k)
            raise
        return {"event": ev, "slot": k, "views": views, "stream": s}

    def poll(self, h) -> bool:
        return h["event"].query()

    def wait_any(self, handles):
        if handles:
            handles[0]["event"].synchronize()

    def collect(self, h):
        sl = self._s[h["slot"]]
        try:
            h["event"].synchronize()
            self.ctx.status(h["stream"])
            h_out = sl["h_out"].numpy()
            res = []
            for i, v in enumerate(h["views"]):
                on, n, g = v["N"]
                N = h_out[on:on + n * g * 4].view(np.int32).reshape(n, g).copy()
                hist = None
                if "hist" in v:
                    ok, oc, g = v["hist"]
                    L = int(sl["h_len"][i])
                    keys = sl["dev"][ok:ok + L * g * 4].view(self.torch.int32).view(L, g).cpu().numpy()
                    cnt = sl["dev"][oc:oc + L * 8].view(self.torch.int64).cpu().numpy().astype(np.uint64)
                    hist = (keys, cnt)
                res.append((N, hist))
            return res
        finally:
            self._free.append(h["slot"])


def poisson_requests(rate: float, count: int, seed: int, max_log2: int = 20):
    """Request shapes of the serving workload: arrival gaps exponential with
    the given rate; n = floor(2^(max_log2 * U)); g uniform in {2, 3, 4}; q
    uniform over the odd prime powers below 300, 50 and 15 for g = 2, 3, 4."""
    rng = np.random.default_rng(seed)
    qs = {2: [q for q in range(3, 300) if odd_prime_power(q)],
          3: [q for q in range(3, 50) if odd_prime_power(q)],
          4: [q for q in range(3, 15) if odd_prime_power(q)]}
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        g = int(rng.integers(2, 5))
        q = int(qs[g][rng.integers(0, len(qs[g]))])
        n = int(2 ** (max_log2 * rng.random()))
        out.append((t, q, g, n, int(rng.integers(0, 2 ** 31))))
    return out


def percentile(vals, p):
    if not vals:
        return None
    return float(np.percentile(np.asarray(vals), p))


def serve_bench(ctx, rates=(0.25, 0.5, 0.75, 0.9), requests: int = 120, seed: int = 180511995,
                batch_curves: int = 1 << 22, max_log2: int = 20, log=print) -> dict:
    """Capacity with every request queued at t = 0, then Poisson arrivals at
    fractions of that capacity; curves/s and p50/p99 latency per rate."""
    from . import curvegen
    ex = GpuExecutor(ctx, batch_curves=batch_curves)

    def make(shapes):
        reqs = []
        for i, (t, q, g, n, s) in enumerate(shapes):
            reqs.append(Request(i, q, g, curvegen.sample(q, g, n, seed=s), arrival=t))
        return reqs

    shapes = poisson_requests(1.0, requests, seed, max_log2)
    # warm the table cache and the kernels, then measure capacity
    warm = Server(ex, batch_curves)
    for r in make(shapes[:8]):
        warm.submit(r)
    warm.drain()
    reqs = make(shapes)
    srv = Server(ex, batch_curves)
    t0 = time.perf_counter()
    for r in reqs:
        r.arrival = t0
        srv.submit(r)
    srv.drain()
    wall = time.perf_counter() - t0
    cap_req = len(reqs) / wall
    cap_curves = sum(r.n for r in reqs) / wall
    fails = sum(1 for r in reqs if r.error)
    log(f"capacity: {cap_req:.1f} req/s, {cap_curves:.4g} curves/s ({fails} failed)")
    out = {"capacity_req_per_s": round(cap_req, 2), "capacity_curves_per_s": round(cap_curves, 1),
           "requests": len(reqs), "rates": []}
    for f in rates:
        lam = f * cap_req
        shp = poisson_requests(lam, requests, seed + int(100 * f), max_log2)
        reqs = make(shp)
        srv = Server(ex, batch_curves)
        t0 = time.perf_counter()
        i = 0
        while i < len(reqs) or srv.pending or srv.inflight:
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                reqs[i].arrival += t0
                srv.submit(reqs[i])
                i += 1
            if not srv.step():
                if srv.inflight:
                    ex.poll(srv.inflight[0][0])
                time.sleep(0.0002)
        wall = time.perf_counter() - t0
        lat = [r.latency for r in reqs if r.error is None]
        row = {"load": f, "arrival_req_per_s": round(lam, 2), "curves_per_s": round(sum(r.n for r in reqs) / wall, 1),
               "p50_ms": round(1e3 * percentile(lat, 50), 3), "p99_ms": round(1e3 * percentile(lat, 99), 3),
               "batches": srv.batches, "failed": sum(1 for r in reqs if r.error)}
        log(f"load {f}: {row}")
        out["rates"].append(row)
    out["cache"] = ctx.stats()
    return out


if __name__ == "__main__":
    import json
    import sys
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_1805_11991_amd import hwcount
    print(json.dumps(serve_bench(hwcount.Context(device=0))))
