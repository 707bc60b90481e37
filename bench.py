#!/usr/bin/env python3
"""Throughput of the Hasse-Weil curve counter on one MI355X.

One step = one pass of the whole path over one batch resident in HBM: curve
bucketing by zero pattern, the count of N_1..N_g for every curve (Zech-table
kernel, persistent and fused over all levels), and the sorted histogram of the
tuples.  Workload of `value`: g = 3 over F_13, 2^24 seeded square-free curves
(the set the metric is quoted on), Frobenius-orbit sweep, graph replay.

Also measured in the same run: the plain form (one launch per level plus a
separate assembly, no graph) on the same set, both forms with the full sweep,
the g = 4 / F_13 set of 2^26 curves in both forms, a profiled loop that times
the count kernel with HIP events on its launch stream (roofline), and the CPU
oracle on a bounded sample (cpu_baseline).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LDS_BANKS_PER_CU = 32          # u16 gathers served per clock per CU without conflicts
NUM_CU = 256
CLOCK_HZ = 2.4e9
LDS_PEAK_LOOKUPS = LDS_BANKS_PER_CU * NUM_CU * CLOCK_HZ
# one wave64 vector ALU instruction per CU per clock (four SIMDs of 16 lanes)
VALU_PEAK_OPS = 64 * NUM_CU * CLOCK_HZ
MFMA_INT8_PEAK_OPS = 5.0e15   # dense int8 matrix-core peak
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "count_kernel_g3_q13_2p24_hbm_traffic.md")
KERNEL_SOURCES = ("paper_1805_11991_amd/csrc/kernels.hip", "paper_1805_11991_amd/csrc/vcount.hip",
                  "paper_1805_11991_amd/csrc/plan.h",
                  "paper_1805_11991_amd/autotune/gfx950.json")


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def lookups_per_batch(curves, levels: list[dict]) -> tuple[int, int]:
    """Table reads the count kernel's algorithm needs for a batch, and the
    plain-Horner count for reference.

    Plain Horner: one read per nonzero term below the leading one, for every
    swept x.  Split evaluation (levels with msplit = m): a tuple of m points
    costs sum_r (terms of class r - 1) reads for the sub-polynomials plus the
    combinations, m (m - 1) for m = 2, 3 (chained) and 8 for m = 4 (two
    radix-2 stages), when every class holds a term; other rows and the single
    points cost plain Horner.  Recomputations on vanishing bases are not
    counted."""
    import numpy as np
    sup = curves.astype(np.int64) != 0
    terms = sup.sum(axis=1)
    horner = terms - 1
    total = plain = 0
    for L in levels:
        plain += int(horner.sum()) * L["nx"]
        m = L["msplit"]
        if not m:
            total += int(horner.sum()) * L["nx"]
            continue
        cls = [sup[:, r::m].sum(axis=1) for r in range(m)]
        ok = np.logical_and.reduce([cc > 0 for cc in cls])
        per_tuple = sum(cc - 1 for cc in cls) + (8 if m == 4 else m * (m - 1))
        cost = np.where(ok, L["nt"] * per_tuple + L["ns"] * horner, L["nx"] * horner)
        total += int(cost.sum())
    return total, plain


def mfma_work(n: int, levels: list[dict]) -> dict:
    """Work of the matrix-core count kernel for n curves.  Every level j
    (k = j coordinates) evaluates each curve at its swept points, padded to
    blocks of 32: one int8 product of K = 16 per coordinate and point (the
    matrix cores), and per (curve, point) pair 4k vector ALU operations: for
    each coordinate its residue (multiply and shift for the quotient, then
    multiply-adds into the table index; coordinate 0 arrives with the table
    offset already added, one multiply-add fewer) and one add of the
    character read.  In the balanced form (mfma = 2) the quotient of every
    coordinate but the first is one multiply-high: 3k + 1 operations."""
    tiles = (n + 31) // 32
    pairs = valu = mfma = 0
    for j, L in enumerate(levels, start=1):
        pts = (L["nx"] + 31) // 32 * 32
        pr = tiles * 32 * pts
        pairs += pr
        valu += pr * ((3 * j + 1) if L["mfma"] == 2 else 4 * j)
        mfma += pr * j * 16 * 2
    return {"pairs": pairs, "valu_ops": valu, "mfma_ops": mfma}


def evaluated_rows(ctx, q: int, g: int, d_rows):
    """The rows the count kernel evaluates for d_rows (rows with zero
    coefficients replaced by their dense translates), on the host."""
    import torch
    out = torch.empty_like(d_rows)
    ctx.translate_dev(q, g, d_rows, out)
    ctx.status()
    return out.cpu().numpy()


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        path = os.path.join(ROOT, rel)
        if os.path.exists(path):
            with open(path, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic() -> dict | None:
    """HBM bytes per launch of the count kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's
    reading for a copy of known size); None when the kernel sources have
    changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    vals = {}
    with open(TRAFFIC_SUMMARY) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256_16") != kernel_source_hash():
        return None
    try:
        return {"fetch": int(vals["fetch_bytes_per_launch"]), "write": int(vals["write_bytes_per_launch"])}
    except (KeyError, ValueError):
        return None


def calibration_copy(torch, dev, nbytes: int = 1 << 30, reps: int = 3):
    """A plain copy kernel of known size (nbytes read, nbytes written) whose
    FETCH_SIZE / WRITE_SIZE readings scale the count kernel's."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    log(f"calibration copy: {reps} x {nbytes} bytes read and written")


def time_loop(fn, steps: int, warmup: int, sync) -> float:
    for _ in range(warmup):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--quick", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB copy kernel (scale for the traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the counter has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1805_11991_amd import curvegen, hwcount

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    sync = torch.cuda.synchronize
    ctx = hwcount.Context(device=0)

    def setup(q, g, n, seed):
        t0 = time.perf_counter()
        curves = curvegen.sample(q, g, n, seed=seed)
        log(f"generated q={q} g={g} n={n} in {time.perf_counter() - t0:.1f}s")
        d = torch.from_numpy(curves).to(dev)
        N = torch.empty((n, g), dtype=torch.int32, device=dev)
        hk = torch.empty((n, g), dtype=torch.int32, device=dev)
        hc = torch.empty(n, dtype=torch.int64, device=dev)
        hl = torch.zeros(1, dtype=torch.int64, device=dev)
        return curves, d, N, hk, hc, hl

    def runner(q, g, bufs, flags):
        _, d, N, hk, hc, hl = bufs
        return lambda: ctx.count_curves_dev(q, g, d, N, hk, hc, hl, flags=flags, stream=stream)

    # ---------------- headline: g = 3, q = 13, 2^24 curves ----------------
    q, g, n = 13, 3, 1 << 24
    bufs = setup(q, g, n, curvegen.BASE_SEED + 1)
    curves = bufs[0]
    batched = runner(q, g, bufs, 0)
    ms = time_loop(batched, args.steps, args.warmup, sync) * 1e3
    ctx.status()
    value = n / (ms * 1e-3)
    log(f"g3 q13 batched orbit: {ms:.3f} ms/step, {value:.4g} curves/s")
    Nref = bufs[2].cpu().numpy()
    nhist = int(bufs[5].item())

    # roofline: the count kernel timed with HIP events on its launch stream
    ctx.profile(True)
    for _ in range(args.steps):
        batched()
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.status()
    assert np.array_equal(bufs[2].cpu().numpy(), Nref), "profiled run differs from the graph run"
    count_ms = prof["count_ms"] / prof["calls"]
    levels = ctx.plan_info(q, g)
    nx = [L["nx"] for L in levels]
    traffic = measured_traffic()
    common = {
        "traffic": None if traffic is None else traffic["fetch"] + traffic["write"],
        "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "traffic_detail": traffic,
        "kernel_ms": round(count_ms, 4),
        "prep_ms": round(prof["prep_ms"] / prof["calls"], 4),
        "hist_ms": round(prof["hist_ms"] / prof["calls"], 4),
    }
    if levels[0]["mfma"]:
        # matrix-core path: bound by the vector ALU work on the products
        work = mfma_work(n, levels)
        achieved = work["valu_ops"] / (count_ms * 1e-3)
        mfma_rate = work["mfma_ops"] / (count_ms * 1e-3)
        roofline = {
            "bound": "alu",
            "achieved": round(achieved / 1e9, 1),
            "peak": round(VALU_PEAK_OPS / 1e9, 1),
            "unit": "G int32 lane-ops/s",
            "frac": round(achieved / VALU_PEAK_OPS, 4),
            **common,
            "kernel": "vcount_kernel<3,int8>",
            "pairs_per_launch": work["pairs"],
            "valu_ops_per_launch": work["valu_ops"],
            "mfma_int8_ops_per_launch": work["mfma_ops"],
            "mfma_int8_tops": round(mfma_rate / 1e12, 2),
            "mfma_frac": round(mfma_rate / MFMA_INT8_PEAK_OPS, 4),
            "levels": [{"M": L["M"], "nx": L["nx"], "pts_padded": (L["nx"] + 31) // 32 * 32} for L in levels],
        }
        log(f"roofline: count kernel {count_ms:.3f} ms, {work['pairs'] / (count_ms * 1e-3) / 1e9:.0f} G "
            f"(curve, point) pairs/s, {achieved / 1e12:.2f} T lane-ops/s ({achieved / VALU_PEAK_OPS:.3f} of "
            f"the vector ALU peak), int8 MFMA {mfma_rate / 1e12:.1f} TOPS ({mfma_rate / MFMA_INT8_PEAK_OPS:.4f})")
    else:
        # the rows the kernel evaluates: zero-coefficient rows become dense translates
        lookups, plain_lookups = lookups_per_batch(evaluated_rows(ctx, q, g, bufs[1]), levels)
        achieved = lookups / (count_ms * 1e-3)
        roofline = {
            "bound": "lds",
            "achieved": round(achieved / 1e9, 2),
            "peak": round(LDS_PEAK_LOOKUPS / 1e9, 1),
            "unit": "Glookup/s",
            "frac": round(achieved / LDS_PEAK_LOOKUPS, 4),
            **common,
            "kernel": "count_kernel<3,int8>",
            "lookups_per_launch": lookups,
            "plain_horner_lookups": plain_lookups,
            "levels": [{k: L[k] for k in ("M", "form", "nx", "msplit", "nt", "ns")} for L in levels],
        }
        # the practical ceiling of that bound on this device: a kernel doing
        # nothing but dependent random reads of a table the size of the top level's
        ceiling = ctx.lds_gather_rate(2 * (q ** g - 1), chains=4)
        roofline["gather_ceiling"] = round(ceiling / 1e9, 2)
        roofline["frac_of_gather_ceiling"] = round(achieved / ceiling, 4)
        log(f"roofline: count kernel {count_ms:.3f} ms, {achieved / 1e9:.1f} Glookup/s "
            f"({achieved / LDS_PEAK_LOOKUPS:.3f} of LDS peak, {achieved / ceiling:.3f} of the "
            f"measured gather ceiling {ceiling / 1e9:.0f} Glookup/s)")

    extra = {}
    if not args.quick:
        for name, flags in (("plain_orbit", hwcount.HWC_PLAIN), ("batched_full", hwcount.HWC_FULL_SWEEP),
                            ("plain_full", hwcount.HWC_PLAIN | hwcount.HWC_FULL_SWEEP)):
            fn = runner(q, g, bufs, flags)
            m = time_loop(fn, max(1, min(args.steps, 3)), 1, sync) * 1e3
            ctx.status()
            assert np.array_equal(bufs[2].cpu().numpy(), Nref), f"{name} differs from batched"
            assert int(bufs[5].item()) == nhist
            extra[name] = {"ms_per_step": round(m, 3), "curves_per_s": round(n / (m * 1e-3), 1)}
            log(f"g3 q13 {name}: {m:.3f} ms/step")
        extra["batched_vs_plain"] = round(extra["plain_orbit"]["ms_per_step"] / ms, 3)
        # counts plus the factorization partition lambda and the (N, lambda)
        # histogram (the full map of eq. 1.2)
        lam = torch.empty(n, dtype=torch.int32, device=dev)
        hk1 = torch.empty((n, g + 1), dtype=torch.int32, device=dev)
        _, d, N, _, hc, hl = bufs

        def with_lambda():
            ctx.count_lambda_dev(q, g, d, N, lam, hk1, hc, hl, stream=stream)
        ml = time_loop(with_lambda, max(1, min(args.steps, 3)), 1, sync) * 1e3
        ctx.status()
        assert np.array_equal(N.cpu().numpy(), Nref), "lambda mode changed N"
        extra["with_lambda"] = {"ms_per_step": round(ml, 3), "curves_per_s": round(n / (ml * 1e-3), 1),
                                "histogram_distinct": int(hl.item())}
        log(f"g3 q13 with lambda: {ml:.3f} ms/step ({int(hl.item())} distinct (N, lambda))")
        del lam, hk1
        # host buffers through the synchronous entry point: PCIe copies of the
        # codes, N and the histogram included (never the headline value)
        Nh = None
        curves16 = curves.astype(np.int16)          # the host entry point takes int16 codes
        t0 = time.perf_counter()
        for _ in range(2):
            Nh, _hist = ctx.count_curves(q, g, curves16, hist_capacity=n)
        mh = (time.perf_counter() - t0) / 2 * 1e3
        assert np.array_equal(Nh, Nref), "host-buffer path differs"
        extra["host_buffers"] = {"ms_per_step": round(mh, 3), "curves_per_s": round(n / (mh * 1e-3), 1)}
        log(f"g3 q13 host buffers (PCIe included): {mh:.3f} ms/step")
        del bufs
        torch.cuda.empty_cache()
        # ---------------- g = 4, q = 13, 2^26 curves ----------------
        n4 = 1 << 26
        bufs4 = setup(13, 4, n4, curvegen.BASE_SEED + 3)
        g4 = {}
        steps4 = max(1, min(args.steps, 3))
        for name, flags in (("batched_orbit", 0), ("plain_orbit", hwcount.HWC_PLAIN)):
            fn = runner(13, 4, bufs4, flags)
            m = time_loop(fn, steps4, 1, sync) * 1e3
            ctx.status()
            g4[name] = {"ms_per_step": round(m, 3), "curves_per_s": round(n4 / (m * 1e-3), 1)}
            log(f"g4 q13 {name}: {m:.3f} ms/step")
        g4["batched_vs_plain"] = round(g4["plain_orbit"]["ms_per_step"] / g4["batched_orbit"]["ms_per_step"], 3)
        ctx.profile(True)
        runner(13, 4, bufs4, 0)()
        p4 = ctx.profile_read()
        ctx.profile(False)
        lv4 = ctx.plan_info(13, 4)
        g4["count_kernel_ms"] = round(p4["count_ms"], 3)
        if lv4[0]["mfma"]:
            w4 = mfma_work(n4, lv4)
            g4["path"] = "matrix cores (top level over several passes)"
            g4["valu_ops_per_s"] = round(w4["valu_ops"] / (p4["count_ms"] * 1e-3), 1)
            g4["valu_frac"] = round(w4["valu_ops"] / (p4["count_ms"] * 1e-3) / VALU_PEAK_OPS, 4)
        else:
            lk4, _ = lookups_per_batch(evaluated_rows(ctx, 13, 4, bufs4[1]), lv4)
            g4["path"] = "Zech logarithms"
            g4["glookup_per_s"] = round(lk4 / (p4["count_ms"] * 1e-3) / 1e9, 2)
            g4["lds_frac"] = round(lk4 / (p4["count_ms"] * 1e-3) / LDS_PEAK_LOOKUPS, 4)
        g4["curves"] = n4
        extra["g4_q13"] = g4
        del bufs4
        torch.cuda.empty_cache()

    if not args.quick:
        # the whole map N_{3,13} of eq. (1.2) by Algorithm 1 (reduced representatives)
        t0 = time.perf_counter()
        mk, mc, mreps = ctx.count_map(13, 3)
        mt = time.perf_counter() - t0
        total = 12 * (13 ** 8 - 13 ** 7) + 12 * (13 ** 7 - 13 ** 6)
        assert int(mc.sum()) == total
        extra["map_g3_q13"] = {"seconds": round(mt, 3), "representatives": mreps, "curves_covered": total,
                               "entries": int(len(mk)), "curves_covered_per_s": round(total / mt, 1)}
        log(f"map N_(3,13): {mt:.3f} s, {mreps} representatives for {total} curves, {len(mk)} entries")

    if not args.quick:
        # Table 1 (Sec. 4): one curve over F_{p^2}, lane per x; the paper's K80
        # evaluation times are printed beside for context only
        k80_eval_ms = {101: 0.36, 211: 1.47, 307: 3.11, 401: 0.95, 503: 1.25, 1009: 2.93, 1511: 394.0,
                       2003: 11.5, 3001: 15.4}
        curve = [17, 12, 16, 11, 10, 13, 12]
        rows = []
        for p, k80 in k80_eval_ms.items():
            row = np.array([c % p for c in curve], dtype=np.int16)
            t0 = time.perf_counter()
            Nf, tf = ctx.count_single(p, 2, row, 2, flags=hwcount.HWC_FULL_SWEEP)   # builds the tables
            first = (time.perf_counter() - t0) * 1e3
            Nf, tf = ctx.count_single(p, 2, row, 2, flags=hwcount.HWC_FULL_SWEEP)
            No, to = ctx.count_single(p, 2, row, 2)
            assert Nf.tolist() == No.tolist()
            rows.append({"p": p, "N1": int(Nf[0]), "N2": int(Nf[1]), "first_call_ms": round(first, 2),
                         "kernel_ms_full_sweep": round(tf["kernel_ms"], 4),
                         "kernel_ms_orbit_sweep": round(to["kernel_ms"], 4), "paper_k80_eval_ms": k80})
            log(f"table 1 p={p}: N2={int(Nf[1])} kernels {tf['kernel_ms']:.3f} ms full, "
                f"{to['kernel_ms']:.3f} ms orbits (first call {first:.0f} ms with tables)")
        extra["table1_single_curve"] = rows

    if args.calib_copy:
        calibration_copy(torch, dev)

    cpu = None
    if not args.no_cpu:
        import oracle
        threads = min(os.cpu_count() or 1, 16)
        sample = 1 << 18
        t0 = time.perf_counter()
        ref = oracle.count_curves(q, g, curves[:sample], threads=threads)
        dt = time.perf_counter() - t0
        assert np.array_equal(ref, Nref[:sample]), "oracle disagrees with the GPU on the CPU sample"
        cpu = {"value": round(sample / dt, 1), "unit": "curves/s", "cores": threads, "kind": "oracle",
               "sample": f"first {sample} curves of the g=3 q=13 set, all k=1..3 ({dt:.1f} s)"}
        log(f"cpu oracle: {sample / dt:.1f} curves/s on {threads} threads")

    out = {
        "metric": "curves/s (all k) at g=3 q=13 and g=4 q=13; batched vs plain, bit-exact",
        "value": round(value, 1),
        "unit": "curves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic: seeded uniform square-free curves (SplitMix64/Lemire rejection), no dataset",
        "config": {"workload": "g3_q13_2^24_curves_batched_orbit_sweep", "q": q, "g": g, "curves": n,
                   "levels_nx": nx, "histogram_distinct": nhist},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
