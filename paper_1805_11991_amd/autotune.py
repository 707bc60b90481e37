"""Autotuner for the count kernel's launch and table-placement choices.

For a (q, g, sweep) it times every candidate of the search space on a seeded
sample of curves (HIP events around the count kernel, through the library's
profiling API), requires every candidate to produce bit-identical N, and keeps
the fastest.  Results live in a JSON database keyed by "q,g,sweep" per GPU
architecture (``autotune/<arch>.json`` next to this file); ``Context`` applies
the database's entries as per-plan options when it is created.

    python -m paper_1805_11991_amd.autotune --qg 13,3 --qg 13,4 [--n 1048576] [--out path]

Search space (library options, see include/hwcount.h):
  mfma            only with --with-mfma: the opt-in int8 matrix-product counting (prime
                  q <= 31, image in LDS) against Zech logarithms; without it the
                  database keeps the Zech-logarithm path and sets no mfma option
  split           split evaluation over m-th roots of unity on LDS levels (on/off)
  split_min_m     smallest level (nonzero elements) that is split
  block           threads per workgroup of the count kernel (256, 512, 1024)
  waves_per_simd  register budget of the kernel build (1: free, 6; the 8-wave build
                  spills registers to scratch at g = 3 and 4 and is left out)
  device_tables   which levels' Zech tables sit in device memory instead of LDS
                  (none, the top level, all)
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DB_DIR = os.path.join(HERE, "autotune")

SPACE = {
    "split": [1, 0],
    "split_min_m": [0, 64, 2048],    # 0: every level split, the base field included
    "block": [256, 512, 1024],
    "waves_per_simd": [1, 6],
    "device_tables": ["none", "top"],
}


SMALL_SPACE = {
    "split": [1, 0],
    "block": [256, 512, 1024],
}


def _device_mask(choice, g: int) -> int:
    return {"none": 0, "top": 1 << (g - 1), "all": (1 << g) - 1}[choice] if isinstance(choice, str) else int(choice)


def _opt_ids():
    from . import hwcount as hw
    return {"mfma": hw.HWC_OPT_MFMA, "split": hw.HWC_OPT_SPLIT, "split_min_m": hw.HWC_OPT_SPLIT_MIN_M,
            "block": hw.HWC_OPT_BLOCK,
            "waves_per_simd": hw.HWC_OPT_WAVES_PER_SIMD, "device_tables": hw.HWC_OPT_DEVICE_TABLES}


def db_path(arch: str = "gfx950") -> str:
    return os.path.join(DB_DIR, f"{arch}.json")


def db_key(q: int, g: int, flags: int = 0) -> str:
    from . import hwcount as hw
    return f"{q},{g},{'full' if flags & hw.HWC_FULL_SWEEP else 'orbit'}"


def load_db(path: str | None = None) -> dict:
    path = path or db_path()
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh).get("entries", {})


def apply_db(ctx, db: dict) -> int:
    """Set every entry of db as per-plan options on ctx; returns the count."""
    from . import hwcount as hw
    ids = _opt_ids()
    n = 0
    for key, ent in db.items():
        q, g, sweep = key.split(",")
        flags = hw.HWC_FULL_SWEEP if sweep == "full" else 0
        for name, val in ent["options"].items():
            if name == "device_tables":
                val = _device_mask(val, int(g))
            ctx.set_plan_option(int(q), int(g), ids[name], int(val), flags)
        n += 1
    return n


def tune(ctx, q: int, g: int, n: int = 1 << 20, seed: int = 4711, flags: int = 0, reps: int = 3,
         space: dict | None = None, log=print) -> dict:
    """Time every candidate; return {"options", "count_ms", "table"}."""
    import numpy as np
    import torch

    from . import curvegen
    from . import hwcount as hw

    space = space or SPACE
    ids = _opt_ids()
    curves = curvegen.sample(q, g, n, seed=seed)
    d = torch.from_numpy(curves).cuda()
    N = torch.empty((n, g), dtype=torch.int32, device="cuda")
    ref = None
    table = []
    names = list(space)
    for values in itertools.product(*(space[k] for k in names)):
        cand = dict(zip(names, values))
        if cand.get("split") == 0 and cand.get("split_min_m", 0) != space.get("split_min_m", [0])[0]:
            continue                      # the threshold means nothing without the split
        if cand.get("mfma") == 1 and any(cand[k] != space[k][0] for k in cand
                                         if k in space and k not in ("mfma", "block")):
            continue                      # only the block size applies to the matrix-core kernel
        try:
            for k, v in cand.items():
                ctx.set_plan_option(q, g, ids[k], _device_mask(v, g) if k == "device_tables" else v, flags)
            ctx.count_curves_dev(q, g, d, N, flags=flags | hw.HWC_NO_GRAPH)   # warm-up, builds the plan
            ctx.status()
            ctx.profile(True)
            for _ in range(reps):
                ctx.count_curves_dev(q, g, d, N, flags=flags)
            prof = ctx.profile_read()
            ctx.profile(False)
            ctx.status()
        except hw.HwcError as e:
            ctx.profile(False)
            log(f"  {cand}: skipped ({e})")
            continue
        got = N.cpu().numpy()
        if ref is None:
            ref = got
        elif not np.array_equal(got, ref):
            raise AssertionError(f"candidate {cand} changed the counts")
        ms = prof["count_ms"] / max(prof["calls"], 1)
        table.append({"options": cand, "count_ms": round(ms, 4)})
        log(f"  {cand}: count kernel {ms:.3f} ms")
    if not table:
        raise RuntimeError(f"no candidate ran for q={q} g={g}")
    best = min(table, key=lambda r: r["count_ms"])
    for k, v in best["options"].items():
        ctx.set_plan_option(q, g, ids[k], _device_mask(v, g) if k == "device_tables" else v, flags)
    return {"options": best["options"], "count_ms": best["count_ms"], "sample": n, "table": table}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--qg", action="append", default=[], help="q,g to tune (repeatable)")
    ap.add_argument("--ranges", action="store_true",
                    help="every (q, g) of the data-production ranges: g=2 q<300, g=3 q<50, g=4 q<15")
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--full-sweep", action="store_true")
    ap.add_argument("--out", default=None)
    ap.add_argument("--arch", default="gfx950")
    ap.add_argument("--with-mfma", action="store_true", help="also try the matrix-product path")
    ap.add_argument("--small", action="store_true",
                    help="reduced space (split, block) for the many small plans of the batched sets")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    from . import hwcount as hw
    flags = hw.HWC_FULL_SWEEP if args.full_sweep else 0
    out = args.out or db_path(args.arch)
    db = {}
    if os.path.exists(out):
        with open(out) as fh:
            db = json.load(fh).get("entries", {})
    ctx = hw.Context(device=0, autotune_db=None)
    todo = list(args.qg)
    if args.ranges:
        from .serving import odd_prime_power
        for g, bound in ((4, 15), (3, 50), (2, 300)):
            todo += [f"{q},{g}" for q in range(3, bound) if odd_prime_power(q)]
    if not todo:
        ap.error("nothing to tune: give --qg or --ranges")
    for qg in todo:
        q, g = (int(v) for v in qg.split(","))
        t0 = time.time()
        # big plans get the whole space; the many small ones the reduced one
        big = q ** g > 20000
        space = dict(SPACE if big and not args.small else SMALL_SPACE)
        if args.with_mfma:
            space = {"mfma": [1, 0], **space}
        n = args.n if big else min(args.n, 1 << 18)
        print(f"tuning q={q} g={g} on {n} curves", flush=True)
        res = tune(ctx, q, g, n=n, flags=flags, space=space)
        print(f"best {res['options']}: {res['count_ms']} ms ({time.time() - t0:.0f} s)", flush=True)
        db[db_key(q, g, flags)] = res
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as fh:
        json.dump({"arch": args.arch, "entries": db}, fh, indent=1)
    print(f"wrote {out}")


if __name__ == "__main__":
    main()
