"""GPU parity: libhwcount.so against the CPU oracle, element by element.

Every per-curve N_k must be bit-exact, and every histogram identical to the
oracle's (sorted distinct tuples and their multiplicities).  Inputs are the
seeded synthetic sets of the workloads: the full enumeration of g=2 over F_5,
slices of the g=3 and g=4 sets over F_13, and sets for other (q, g) including
prime powers.  All four launch forms are checked: the persistent batched
kernel (default), the plain per-level launches, each with the Frobenius-orbit
sweep and with the full sweep.
"""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MODES = {
    "batched-orbit": 0,
    "batched-full": 1,      # HWC_FULL_SWEEP
    "plain-orbit": 2,       # HWC_PLAIN
    "plain-full": 3,
}


@pytest.fixture(scope="module")
def gctx():
    """The default context: Zech-logarithm evaluation on every plan."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_11991_amd import hwcount
    ctx = hwcount.Context(device=0)
    yield ctx
    ctx.close()


@pytest.fixture(scope="module")
def mctx():
    """A context with the opt-in matrix-product path (prime q <= 31)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_11991_amd import hwcount
    ctx = hwcount.Context(device=0, mfma=True)
    yield ctx
    ctx.close()


def _path_of(ctx, q, g):
    """"mfma" when the plan of (q, g) counts by matrix products, else "zech"."""
    return "mfma" if ctx.plan_info(q, g)[0]["mfma"] else "zech"


def _hist_np(N):
    keys, counts = np.unique(N, axis=0, return_counts=True)
    return keys.astype(np.int32), counts.astype(np.uint64)


def _check(gctx, oracle_mod, q, g, curves, modes=MODES, hist=True, Nref=None):
    if Nref is None:
        Nref = oracle_mod.count_curves(q, g, curves)
    kref, cref = oracle_mod.histogram(Nref) if hist else (None, None)
    for name, flags in modes.items():
        print(f"  mode {name} q={q} g={g} n={len(curves)}", flush=True)
        N, H = gctx.count_curves(q, g, curves, flags=flags, hist_capacity=len(curves) if hist else None)
        bad = np.flatnonzero((N != Nref).any(axis=1))
        assert bad.size == 0, (name, q, g, bad[:5], N[bad[:5]], Nref[bad[:5]], curves[bad[:5]])
        if hist:
            assert np.array_equal(H[0], kref), name
            assert np.array_equal(H[1], cref), name
    return Nref


def test_g2_q5_full_enumeration(gctx, oracle_mod, curvegen_mod):
    curves = curvegen_mod.enumerate_all(5, 2)
    assert len(curves) == 60000
    _check(gctx, oracle_mod, 5, 2, curves)


def test_default_path_is_zech(gctx, mctx):
    # the default evaluates with Zech logarithms everywhere; the matrix-product
    # path runs only where it was asked for (and exists: prime q <= 31)
    for q, g in ((13, 3), (13, 4), (5, 2), (7, 4), (9, 3)):
        assert _path_of(gctx, q, g) == "zech", (q, g)
    for q, g in ((13, 3), (13, 4), (5, 2), (7, 4)):
        assert _path_of(mctx, q, g) == "mfma", (q, g)
    assert _path_of(mctx, 9, 3) == "zech"      # prime powers have no matrix-product form


def test_g3_q13_slice(gctx, mctx, oracle_mod, curvegen_mod):
    curves = curvegen_mod.sample(13, 3, 6000, seed=curvegen_mod.BASE_SEED + 1)
    Nref = _check(gctx, oracle_mod, 13, 3, curves)
    _check(mctx, oracle_mod, 13, 3, curves, Nref=Nref)


def test_g4_q13_slice(gctx, mctx, oracle_mod, curvegen_mod):
    curves = curvegen_mod.sample(13, 4, 400, seed=curvegen_mod.BASE_SEED + 3)
    Nref = _check(gctx, oracle_mod, 13, 4, curves)
    _check(mctx, oracle_mod, 13, 4, curves, Nref=Nref)


def test_g4_q3_full_enumeration(gctx, oracle_mod, curvegen_mod):
    curves = curvegen_mod.enumerate_all(3, 4)
    assert len(curves) == 104976
    _check(gctx, oracle_mod, 3, 4, curves, modes={"batched-orbit": 0, "plain-full": 3})


@pytest.mark.parametrize("q,g,n", [
    (3, 1, 200), (7, 1, 300), (101, 1, 300),
    (9, 2, 400), (25, 2, 300), (27, 2, 300), (49, 2, 200), (81, 2, 150), (121, 2, 100), (125, 2, 100),
    (169, 2, 60), (181, 2, 60),
    (3, 3, 500), (5, 3, 400), (7, 3, 300), (9, 3, 200), (11, 3, 200), (17, 3, 60), (25, 3, 30), (31, 3, 20),
    (5, 4, 150), (7, 4, 60), (9, 4, 40), (11, 4, 20),
    # q = 3 mod 4 with top levels in element units or device memory: split over mu_2
    (107, 2, 200), (179, 2, 100), (23, 3, 80), (27, 3, 60), (31, 3, 130), (43, 3, 8), (47, 3, 6), (11, 4, 300),
])
def test_other_fields(gctx, mctx, oracle_mod, curvegen_mod, q, g, n):
    curves = curvegen_mod.sample(q, g, n, seed=4242 + q * 10 + g, dtype=np.int16)
    Nref = _check(gctx, oracle_mod, q, g, curves)
    if _path_of(mctx, q, g) == "mfma":
        _check(mctx, oracle_mod, q, g, curves, Nref=Nref)


@pytest.mark.parametrize("path", ["zech", "mfma"])
def test_sparse_patterns(gctx, mctx, oracle_mod, curvegen_mod, path):
    # rows with many zero coefficients: on the Zech path the masked (gap)
    # Horner sweep with translates off, and the dense translates with them on;
    # on the matrix-product path zeros are zeros of the product
    from paper_1805_11991_amd import hwcount as hw
    ctxs = [mctx] if path == "mfma" else [gctx]
    if path == "zech":
        noshift = hw.Context(device=0, autotune_db=None)
        noshift.set_option(hw.HWC_OPT_SHIFT, 0)
        ctxs.append(noshift)
    rng = np.random.default_rng(5)
    for q, g in ((13, 3), (13, 4), (7, 2)):
        for ctx in ctxs:
            assert _path_of(ctx, q, g) == path
        nc = 2 * g + 3
        rows = []
        while len(rows) < 300:
            r = rng.integers(0, q, size=nc)
            r[rng.random(nc) < 0.6] = 0
            if r[-1] == 0 and r[-2] == 0:
                r[-1] = 1
            if curvegen_mod.is_squarefree(q, r):
                rows.append(r)
        rows.append([1] + [0] * (2 * g) + [1, 0])          # x^{2g+1} + 1
        rows.append([0, 1] + [0] * (2 * g - 1) + [0, 1])   # x^{2g+2} + x
        curves = np.array(rows, dtype=np.int16)
        Nref = oracle_mod.count_curves(q, g, curves)
        for ctx in ctxs:
            _check(ctx, oracle_mod, q, g, curves, Nref=Nref)
    if path == "zech":
        ctxs[1].close()


def test_int8_and_int16_agree(gctx, mctx, oracle_mod, curvegen_mod):
    import torch
    for q, g in ((13, 3), (13, 4)):
        curves = curvegen_mod.sample(q, g, 5000 if g == 3 else 700, seed=77)
        ref = oracle_mod.count_curves(q, g, curves)
        for ctx in (gctx, mctx):
            for dt in (torch.int8, torch.int16):
                d = torch.from_numpy(curves.astype(np.int16)).to(dt).cuda()
                N = torch.empty((len(curves), g), dtype=torch.int32, device="cuda")
                ctx.count_curves_dev(q, g, d, N)
                ctx.status()
                assert np.array_equal(N.cpu().numpy(), ref), (q, g, dt, _path_of(ctx, q, g))


def test_edge_sizes(gctx, mctx, oracle_mod, curvegen_mod):
    for ctx in (gctx, mctx):
        for n in (0, 1, 31, 32, 33, 63, 64, 65, 129):
            curves = curvegen_mod.sample(13, 3, n, seed=9 + n, dtype=np.int16)
            N, H = ctx.count_curves(13, 3, curves, hist_capacity=max(n, 1))
            assert N.shape == (n, 3)
            if n:
                ref = oracle_mod.count_curves(13, 3, curves)
                assert np.array_equal(N, ref), (n, _path_of(ctx, 13, 3))
                k, c = oracle_mod.histogram(ref)
                assert np.array_equal(H[0], k) and np.array_equal(H[1], c)
            else:
                assert len(H[0]) == 0


def test_errors(gctx):
    from paper_1805_11991_amd import hwcount
    good = np.array([[1, 0, 0, 0, 0, 1, 0]], dtype=np.int16)
    cases = [
        (dict(q=15, g=2, coeffs=good), hwcount.HWC_ERR_NOT_ODD_PRIME_POWER),
        (dict(q=5, g=0, coeffs=np.zeros((1, 3), np.int16)), hwcount.HWC_ERR_BAD_G),
        (dict(q=5, g=2, coeffs=np.array([[5, 0, 0, 0, 0, 1, 0]], np.int16)), hwcount.HWC_ERR_COEFF_RANGE),
        (dict(q=5, g=2, coeffs=np.array([[1, 0, 0, 0, 1, 0, 0]], np.int16)), hwcount.HWC_ERR_DEGREE),
        (dict(q=4099, g=2, coeffs=good), hwcount.HWC_ERR_FIELD_TOO_LARGE),   # q^2 > 2^24
    ]
    for kw, code in cases:
        with pytest.raises(hwcount.HwcError) as ei:
            gctx.count_curves(kw["q"], kw["g"], kw["coeffs"])
        assert ei.value.code == code, kw
    # (x+1)^2 (x^3+2) over F_5 has a square factor
    from paper_1805_11991_amd import curvegen
    sing = np.array([[2, 4, 2, 1, 2, 1, 0]], dtype=np.int16)
    assert not curvegen.is_squarefree(5, sing[0])
    with pytest.raises(hwcount.HwcError) as ei:
        gctx.count_curves(5, 2, sing, flags=hwcount.HWC_VALIDATE)
    assert ei.value.code == hwcount.HWC_ERR_SINGULAR
    gctx.count_curves(5, 2, sing)   # without the flag the formula value is returned
    # histogram capacity
    curves = np.array([[1, 0, 0, 0, 0, 1, 0], [2, 0, 0, 0, 0, 1, 0], [1, 1, 0, 0, 0, 1, 0]], np.int16)
    with pytest.raises(hwcount.HwcError) as ei:
        gctx.count_curves(5, 2, curves, hist_capacity=0)
    assert ei.value.code == hwcount.HWC_ERR_HIST_CAPACITY


def test_device_row_errors_reported_by_status(gctx):
    import torch
    from paper_1805_11991_amd import hwcount
    bad = torch.tensor([[7, 0, 0, 0, 0, 1, 0]], dtype=torch.int16, device="cuda")
    N = torch.empty((1, 2), dtype=torch.int32, device="cuda")
    gctx.count_curves_dev(5, 2, bad, N)
    with pytest.raises(hwcount.HwcError) as ei:
        gctx.status()
    assert ei.value.code == hwcount.HWC_ERR_COEFF_RANGE
    gctx.status()   # cleared


def test_graph_replays_match_eager(gctx, curvegen_mod):
    import torch
    from paper_1805_11991_amd import hwcount
    curves = curvegen_mod.sample(13, 3, 20000, seed=31337)
    d = torch.from_numpy(curves).cuda()
    ref = torch.empty((len(curves), 3), dtype=torch.int32, device="cuda")
    gctx.count_curves_dev(13, 3, d, ref, flags=hwcount.HWC_NO_GRAPH)
    hk = torch.empty((len(curves), 3), dtype=torch.int32, device="cuda")
    hc = torch.empty(len(curves), dtype=torch.int64, device="cuda")
    hl = torch.zeros(1, dtype=torch.int64, device="cuda")
    hk0 = torch.empty_like(hk)
    hc0 = torch.empty_like(hc)
    hl0 = torch.zeros_like(hl)
    gctx.count_curves_dev(13, 3, d, ref, hk0, hc0, hl0, flags=hwcount.HWC_NO_GRAPH)
    gctx.status()
    L = int(hl0.item())
    Nrep = torch.empty((len(curves), 3), dtype=torch.int32, device="cuda")
    for rep in range(4):     # first call captures the graph, the rest replay it
        Nrep.fill_(-1)
        hk.fill_(-1)
        hc.fill_(0)
        torch.cuda.synchronize()   # the fills ran on torch's stream, the count runs on the context's
        gctx.count_curves_dev(13, 3, d, Nrep, hk, hc, hl)
        torch.cuda.synchronize()
        _ = (d.float().sum() * 2).item()      # unrelated eager work between replays
        gctx.status()
        assert torch.equal(Nrep, ref), rep
        assert int(hl.item()) == L
        assert torch.equal(hk[:L], hk0[:L]) and torch.equal(hc[:L], hc0[:L])


def test_full_size_g3_q13(gctx, mctx, oracle_mod, curvegen_mod):
    """The 2^24-curve g=3 set over F_13 in the benchmark's launch form
    (persistent, graph, orbit sweep): every N of the Zech path equals the
    matrix-product path's (two independent evaluations), the first 2^18 rows
    and a seeded sample across the whole set equal the oracle's, and the
    device histogram equals the oracle's histogram of N."""
    import torch
    n = 1 << 24
    curves = curvegen_mod.sample(13, 3, n, seed=curvegen_mod.BASE_SEED + 1)
    d = torch.from_numpy(curves).cuda()
    out = {}
    for name, ctx in (("zech", gctx), ("mfma", mctx)):
        assert _path_of(ctx, 13, 3) == name
        N = torch.empty((n, 3), dtype=torch.int32, device="cuda")
        hk = torch.empty((n, 3), dtype=torch.int32, device="cuda")
        hc = torch.empty(n, dtype=torch.int64, device="cuda")
        hl = torch.zeros(1, dtype=torch.int64, device="cuda")
        print(f"  full-size g=3 q=13 on the {name} path", flush=True)
        ctx.count_curves_dev(13, 3, d, N, hk, hc, hl)
        ctx.status()
        L = int(hl.item())
        out[name] = (N.cpu().numpy(), hk[:L].cpu().numpy(), hc[:L].cpu().numpy().astype(np.uint64))
        del N, hk, hc
    Nz, kz, cz = out["zech"]
    Nm, km, cm = out["mfma"]
    bad = np.flatnonzero((Nz != Nm).any(axis=1))
    assert bad.size == 0, (bad[:5], Nz[bad[:5]], Nm[bad[:5]])
    rng = np.random.default_rng(2024)
    idx = np.unique(np.concatenate([np.arange(1 << 18), rng.integers(0, n, 4096), [n - 1]]))
    print(f"  oracle on {len(idx)} rows", flush=True)
    ref = oracle_mod.count_curves(13, 3, curves[idx])
    bad = np.flatnonzero((Nz[idx] != ref).any(axis=1))
    assert bad.size == 0, (idx[bad[:5]], Nz[idx[bad[:5]]], ref[bad[:5]])
    kref, cref = oracle_mod.histogram(Nz)
    for keys, cnt in ((kz, cz), (km, cm)):
        assert np.array_equal(keys, kref) and np.array_equal(cnt, cref)
    assert int(cref.sum()) == n


@pytest.mark.parametrize("q,g,n", [(191, 2, 30), (211, 2, 24), (257, 2, 16), (263, 2, 16), (293, 2, 16), (37, 3, 6),
                                   (41, 3, 5), (43, 3, 4), (49, 3, 3)])
def test_large_level_tables(gctx, oracle_mod, curvegen_mod, q, g, n):
    # 32767 < q^g - 1 <= 65534: one period of u16 entries in LDS (form E);
    # up to 131070: half a period in LDS, as u32 entries where the image fits
    # (form G), else as 17-bit entries (form F)
    curves = curvegen_mod.sample(q, g, n, seed=777 + q, dtype=np.int16)
    top = gctx.plan_info(q, g)[-1]
    assert top["form"] == (3 if q ** g - 1 <= 65534 else 5 if (q, g) in HALF_U32 else 4), top
    _check(gctx, oracle_mod, q, g, curves)


@pytest.mark.parametrize("q,g,n", [(211, 2, 20), (293, 2, 16), (43, 3, 4)])
def test_device_memory_tables(oracle_mod, curvegen_mod, q, g, n):
    """The top level's Zech table placed in device memory (form D, served by
    L2 and the MALL) by the table-placement option."""
    from paper_1805_11991_amd import hwcount as hw
    curves = curvegen_mod.sample(q, g, n, seed=779 + q, dtype=np.int16)
    with hw.Context(device=0, autotune_db=None) as ctx:
        ctx.set_option(hw.HWC_OPT_DEVICE_TABLES, 1 << (g - 1))
        assert ctx.plan_info(q, g)[-1]["form"] == 2
        _check(ctx, oracle_mod, q, g, curves)


# top levels whose u32 half table (4 (M/2 + 1) bytes) fits the LDS image: with
# the levels below (q = 281 at g = 2 leaves under 600 bytes), or once those
# levels are moved to device memory (q = 283 at g = 2, 43 at g = 3)
HALF_U32 = {(257, 2), (263, 2), (269, 2), (271, 2), (277, 2), (281, 2), (283, 2), (41, 3), (43, 3)}
LOWER_IN_DEVICE = {(283, 2), (43, 3)}


@pytest.mark.parametrize("q,g,n", [(289, 2, 20), (293, 2, 20), (47, 3, 5), (49, 3, 4)])
def test_half_period_lds_tables(gctx, oracle_mod, curvegen_mod, q, g, n):
    """Top levels of 65 535 .. 131 070 nonzero elements whose u32 half table
    would not fit: Z(k) for k <= M/2 as 17-bit entries in LDS, the rest through
    Z(-k) = Z(k) - k (form F), split over mu_4 (289, 293, 49) or mu_2 (47), on
    seeded rows and on rows with zero coefficients, every launch form against
    the oracle."""
    assert gctx.plan_info(q, g)[-1]["form"] == 4
    curves = curvegen_mod.sample(q, g, n, seed=780 + q, dtype=np.int16)
    sparse = curves.copy()
    for i in range(len(sparse)):
        top = 2 * g + 2 if sparse[i, 2 * g + 2] else 2 * g + 1
        for k in ((i % top), ((3 * i + 1) % top))[: 1 + i % 2]:
            sparse[i, k] = 0
    _check(gctx, oracle_mod, q, g, curves)
    _check(gctx, oracle_mod, q, g, sparse)


@pytest.mark.parametrize("q,g,n", [(257, 2, 24), (263, 2, 20), (281, 2, 20), (283, 2, 20), (41, 3, 6), (43, 3, 5)])
def test_half_period_u32_lds_tables(gctx, oracle_mod, curvegen_mod, q, g, n):
    """The same half period as u32 entries in byte units (form G, one read per
    lookup, the zero marker folding to itself) where the image fits, with the
    levels below in device memory (form D) where only that makes it fit (283,
    43), split over mu_4 (257, 281, 41) or mu_2 (263, 283, 43), on seeded rows
    and on rows with zero coefficients, every launch form against the oracle."""
    levels = gctx.plan_info(q, g)
    assert (q, g) in HALF_U32 and levels[-1]["form"] == 5
    assert all((L["form"] == 2) == ((q, g) in LOWER_IN_DEVICE) for L in levels[:-1]), levels
    curves = curvegen_mod.sample(q, g, n, seed=781 + q, dtype=np.int16)
    sparse = curves.copy()
    for i in range(len(sparse)):
        top = 2 * g + 2 if sparse[i, 2 * g + 2] else 2 * g + 1
        for k in ((i % top), ((3 * i + 1) % top))[: 1 + i % 2]:
            sparse[i, k] = 0
    _check(gctx, oracle_mod, q, g, curves)
    _check(gctx, oracle_mod, q, g, sparse)


@pytest.mark.parametrize("q,g,n", [(191, 2, 40), (227, 2, 30), (241, 2, 30), (251, 2, 30), (37, 3, 8)])
def test_one_period_lds_tables(gctx, oracle_mod, curvegen_mod, q, g, n):
    """Top levels of 32 768 .. 65 534 nonzero elements: one period of u16 Zech
    entries in LDS (form E), split over mu_4 (241, 37) or mu_2 (191, 227, 251),
    on seeded rows and on rows with zero coefficients (the masked path), every
    launch form against the oracle."""
    assert gctx.plan_info(q, g)[-1]["form"] == 3
    curves = curvegen_mod.sample(q, g, n, seed=778 + q, dtype=np.int16)
    sparse = curves.copy()
    for i in range(len(sparse)):           # zero one or two coefficients below the leading one
        top = 2 * g + 2 if sparse[i, 2 * g + 2] else 2 * g + 1
        for k in ((i % top), ((3 * i + 1) % top))[: 1 + i % 2]:
            sparse[i, k] = 0
    # a zeroed row need not stay square-free: the library and the oracle
    # evaluate the same character sums on any row of that degree
    _check(gctx, oracle_mod, q, g, curves)
    _check(gctx, oracle_mod, q, g, sparse)


def _batch_specs(curvegen_mod):
    specs = []
    specs.append((5, 2, curvegen_mod.enumerate_all(5, 2)[::7]))
    specs.append((13, 3, curvegen_mod.sample(13, 3, 3000, seed=curvegen_mod.BASE_SEED + 1)))
    specs.append((3, 4, curvegen_mod.enumerate_all(3, 4)[::50]))
    specs.append((13, 4, curvegen_mod.sample(13, 4, 90, seed=curvegen_mod.BASE_SEED + 3)))
    specs.append((9, 2, curvegen_mod.sample(9, 2, 500, seed=91)))
    specs.append((293, 2, curvegen_mod.sample(293, 2, 10, seed=92)))
    specs.append((49, 3, curvegen_mod.sample(49, 3, 3, seed=93)))
    specs.append((283, 2, curvegen_mod.sample(283, 2, 8, seed=97)))
    specs.append((7, 1, curvegen_mod.sample(7, 1, 300, seed=94)))
    specs.append((13, 3, curvegen_mod.sample(13, 3, 0, seed=95)))          # empty request
    specs.append((11, 4, curvegen_mod.sample(11, 4, 33, seed=96)))
    return specs


def test_multi_plan_batch(gctx, oracle_mod, curvegen_mod):
    """One persistent launch over requests of different (q, g): every request's
    N and histogram equal the oracle's, with graph capture, replay, the direct
    launch and the full sweep."""
    import torch
    from paper_1805_11991_amd import hwcount
    specs = _batch_specs(curvegen_mod)
    refs = [oracle_mod.count_curves(q, g, c) if len(c) else np.zeros((0, g), np.int32) for q, g, c in specs]
    jobs = []
    for (q, g, c) in specs:
        n = len(c)
        jobs.append(dict(q=q, g=g, d_coeffs=torch.from_numpy(c).cuda(),
                         d_out_N=torch.empty((n, g), dtype=torch.int32, device="cuda"),
                         d_hist_keys=torch.empty((max(n, 1), g), dtype=torch.int32, device="cuda"),
                         d_hist_counts=torch.empty(max(n, 1), dtype=torch.int64, device="cuda"),
                         d_hist_len=torch.zeros(1, dtype=torch.int64, device="cuda")))
    for rep, flags in enumerate((0, 0, 0, hwcount.HWC_NO_GRAPH, hwcount.HWC_FULL_SWEEP)):
        print(f"  batch rep {rep} flags {flags}", flush=True)
        for j in jobs:
            j["d_out_N"].fill_(-1)
            j["d_hist_len"].fill_(-1)
        torch.cuda.synchronize()   # the fills ran on torch's stream, the batch runs on the context's
        gctx.count_batch(jobs, flags=flags)
        gctx.status()
        for (q, g, c), j, ref in zip(specs, jobs, refs):
            N = j["d_out_N"].cpu().numpy()
            assert np.array_equal(N, ref), (rep, q, g)
            L = int(j["d_hist_len"].item())
            if len(c):
                k, cnt = oracle_mod.histogram(ref)
                assert L == len(k)
                assert np.array_equal(j["d_hist_keys"][:L].cpu().numpy(), k)
                assert np.array_equal(j["d_hist_counts"][:L].cpu().numpy().astype(np.uint64), cnt)
            else:
                assert L == 0


@pytest.mark.parametrize("q,g,n", [(293, 2, 3000), (47, 3, 600)])
def test_batch_tile_parts(gctx, oracle_mod, curvegen_mod, q, g, n):
    """A batch job of few tiles over a large top level: each tile's top-level
    sweep is cut into parts whose counts are summed before the tile's last part
    assembles N.  On dense rows and on rows with zero coefficients (the split
    and the unsplit point lists), over several tiles with a ragged last one, N
    of the batch equals the single-request path's on every row, in the
    captured graph, its replays and the direct launch, and the oracle's on a
    sample of rows."""
    import torch
    from paper_1805_11991_amd import hwcount
    dense = curvegen_mod.sample(q, g, n, seed=790 + q, dtype=np.int16)
    sparse = dense[: n // 3].copy()
    for i in range(len(sparse)):
        top = 2 * g + 2 if sparse[i, 2 * g + 2] else 2 * g + 1
        for k in ((i % top), ((3 * i + 1) % top))[: 1 + i % 2]:
            sparse[i, k] = 0
    rows = np.concatenate([dense, sparse])
    m = len(rows)
    d = torch.from_numpy(rows).cuda()
    single = torch.empty((m, g), dtype=torch.int32, device="cuda")
    gctx.count_curves_dev(q, g, d, single)
    gctx.status()
    ref = single.cpu().numpy()
    sample = np.r_[0:20, n - 10:n, m - 20:m]
    assert np.array_equal(ref[sample], oracle_mod.count_curves(q, g, rows[sample]))
    job = dict(q=q, g=g, d_coeffs=d, d_out_N=torch.empty((m, g), dtype=torch.int32, device="cuda"))
    for rep, flags in enumerate((0, 0, 0, hwcount.HWC_NO_GRAPH)):
        print(f"  parts rep {rep} flags {flags}", flush=True)
        job["d_out_N"].fill_(-1)
        torch.cuda.synchronize()
        gctx.count_batch([job], flags=flags)
        gctx.status()
        assert np.array_equal(job["d_out_N"].cpu().numpy(), ref), (rep, q, g)


def test_two_streams_are_ordered(gctx, oracle_mod, curvegen_mod):
    """Calls of one context on different streams share scratch; the library
    orders them, so results stay exact when they are issued back to back."""
    import torch
    a = curvegen_mod.sample(13, 3, 4000, seed=501)
    b = curvegen_mod.sample(7, 4, 300, seed=502)
    ra, rb = oracle_mod.count_curves(13, 3, a), oracle_mod.count_curves(7, 4, b)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    torch.cuda.synchronize()
    Na = torch.empty((len(a), 3), dtype=torch.int32, device="cuda")
    Nb = torch.empty((len(b), 4), dtype=torch.int32, device="cuda")
    for _ in range(3):
        gctx.count_curves_dev(13, 3, da, Na, stream=s1)
        gctx.count_curves_dev(7, 4, db, Nb, stream=s2)
    torch.cuda.synchronize()
    gctx.status()
    assert np.array_equal(Na.cpu().numpy(), ra)
    assert np.array_equal(Nb.cpu().numpy(), rb)


# Zech-logarithm options: each set says mfma 0 so that it runs the Zech
# kernels whatever the default is
ZECH_OPTION_SETS = [
    {"mfma": 0},
    {"mfma": 0, "split": 0},
    {"mfma": 0, "device_tables": 1},          # lowest level only in device memory
    {"mfma": 0, "device_tables": 15},         # every level
    {"mfma": 0, "block": 1024, "waves_per_simd": 8},
    {"mfma": 0, "block": 512, "waves_per_simd": 6, "split": 0},
    {"mfma": 0, "split_min_m": 0},            # every level split, down to F_q (vanishing bases everywhere)
    {"mfma": 0, "split_min_m": 2048},
    {"mfma": 0, "block": 1024, "waves_per_simd": 6},
    {"mfma": 0, "shift": 0},                  # rows counted as given (masked Horner on sparse rows)
]
# the matrix-product path's options (only the block size applies)
MFMA_OPTION_SETS = [
    {"mfma": 1},
    {"mfma": 1, "block": 256},
    {"mfma": 1, "block": 512},
    {"mfma": 1, "block": 1024},
]


def _run_option_set(oracle_mod, curvegen_mod, q, g, n, opts, seed, want_path):
    from paper_1805_11991_amd import hwcount as hw
    ids = {"split": hw.HWC_OPT_SPLIT, "block": hw.HWC_OPT_BLOCK, "waves_per_simd": hw.HWC_OPT_WAVES_PER_SIMD,
           "device_tables": hw.HWC_OPT_DEVICE_TABLES, "split_min_m": hw.HWC_OPT_SPLIT_MIN_M,
           "mfma": hw.HWC_OPT_MFMA, "shift": hw.HWC_OPT_SHIFT}
    ctx = hw.Context(device=0, autotune_db=None)
    try:
        for k, v in opts.items():
            ctx.set_plan_option(q, g, ids[k], v)
            ctx.set_plan_option(q, g, ids[k], v, hw.HWC_FULL_SWEEP)
        assert _path_of(ctx, q, g) == want_path, (q, g, opts)
        curves = curvegen_mod.sample(q, g, n, seed=seed)
        Nref = oracle_mod.count_curves(q, g, curves)
        _check(ctx, oracle_mod, q, g, curves, modes={"batched-orbit": 0, "batched-full": 1, "plain-orbit": 2},
               Nref=Nref)
        # the same rows as int16 codes through the device entry point
        import torch
        d = torch.from_numpy(curves.astype(np.int16)).cuda()
        N = torch.empty((n, g), dtype=torch.int32, device="cuda")
        ctx.count_curves_dev(q, g, d, N)
        ctx.status()
        assert np.array_equal(N.cpu().numpy(), Nref)
    finally:
        ctx.close()


@pytest.mark.parametrize("q,g,n", [(13, 3, 3000), (13, 4, 1500), (5, 4, 3000), (9, 3, 2000), (11, 3, 1500),
                                   (7, 3, 2000)])
@pytest.mark.parametrize("opts", range(len(ZECH_OPTION_SETS)))
def test_zech_options_keep_results(oracle_mod, curvegen_mod, q, g, n, opts):
    """Every tunable of the Zech path (split and its threshold, device-memory
    placement of any level's table, block size, register budget, dense
    translates) gives the oracle's counts, and the Zech kernels are what ran."""
    _run_option_set(oracle_mod, curvegen_mod, q, g, n, ZECH_OPTION_SETS[opts], 900 + opts, "zech")


@pytest.mark.parametrize("q,g,n", [(13, 3, 3000), (13, 4, 1500), (5, 4, 3000), (7, 2, 3000), (31, 3, 300)])
@pytest.mark.parametrize("opts", range(len(MFMA_OPTION_SETS)))
def test_mfma_options_keep_results(oracle_mod, curvegen_mod, q, g, n, opts):
    """The matrix-product path at every block size, with one pass holding all
    levels (g = 3, q = 5 at g = 4) or the top level over several passes
    (g = 4, q = 13), int8 and int16 codes."""
    _run_option_set(oracle_mod, curvegen_mod, q, g, n, MFMA_OPTION_SETS[opts], 950 + opts, "mfma")


def test_full_size_g4_q13(gctx, mctx, oracle_mod, curvegen_mod):
    """The 2^26-curve g=4 set over F_13 in the benchmark's launch form: every
    N of the Zech path equals the matrix-product path's, the first 4096 rows
    and a seeded sample equal the oracle's, and the device histogram equals
    the oracle's histogram of N."""
    import torch
    n = 1 << 26
    curves = curvegen_mod.sample(13, 4, n, seed=curvegen_mod.BASE_SEED + 3)
    d = torch.from_numpy(curves).cuda()
    Ns = {}
    hist = None
    for name, ctx in (("zech", gctx), ("mfma", mctx)):
        assert _path_of(ctx, 13, 4) == name
        N = torch.empty((n, 4), dtype=torch.int32, device="cuda")
        print(f"  full-size g=4 q=13 on the {name} path", flush=True)
        if name == "zech":
            hk = torch.empty((n, 4), dtype=torch.int32, device="cuda")
            hc = torch.empty(n, dtype=torch.int64, device="cuda")
            hl = torch.zeros(1, dtype=torch.int64, device="cuda")
            ctx.count_curves_dev(13, 4, d, N, hk, hc, hl)
            ctx.status()
            L = int(hl.item())
            hist = (hk[:L].cpu().numpy(), hc[:L].cpu().numpy().astype(np.uint64))
            del hk, hc
        else:
            ctx.count_curves_dev(13, 4, d, N)
            ctx.status()
        Ns[name] = N.cpu().numpy()
        del N
    bad = np.flatnonzero((Ns["zech"] != Ns["mfma"]).any(axis=1))
    assert bad.size == 0, (bad[:5], Ns["zech"][bad[:5]], Ns["mfma"][bad[:5]])
    rng = np.random.default_rng(4096)
    idx = np.unique(np.concatenate([np.arange(4096), rng.integers(0, n, 512), [n - 1]]))
    print(f"  oracle on {len(idx)} rows", flush=True)
    ref = oracle_mod.count_curves(13, 4, curves[idx])
    assert np.array_equal(Ns["zech"][idx], ref)
    kref, cref = oracle_mod.histogram(Ns["zech"])
    assert np.array_equal(hist[0], kref) and np.array_equal(hist[1], cref)
    assert int(cref.sum()) == n


def _odd_prime_powers_below(bound):
    out = []
    for q in range(3, bound, 2):
        p = next(f for f in range(3, q + 1, 2) if q % f == 0)
        r = q
        while r % p == 0:
            r //= p
        if r == 1:
            out.append(q)
    return out


def test_batch_all_fields_below_300_g2_sampled(gctx, oracle_mod, curvegen_mod):
    """All 71 odd prime powers q < 300 at g = 2, 2^16 curves each, in one
    multi-plan persistent launch (tables in LDS for small q, in device memory
    beyond 2^15 elements); sampled rows against the oracle, every job's
    histogram total and order."""
    import torch
    qs = _odd_prime_powers_below(300)
    assert len(qs) == 71
    n = 1 << 16
    jobs, sets = [], []
    for q in qs:
        c = curvegen_mod.sample(q, 2, n, seed=curvegen_mod.BASE_SEED + 2 + q)
        sets.append(c)
        jobs.append(dict(q=q, g=2, d_coeffs=torch.from_numpy(c).cuda(),
                         d_out_N=torch.empty((n, 2), dtype=torch.int32, device="cuda"),
                         d_hist_keys=torch.empty((n, 2), dtype=torch.int32, device="cuda"),
                         d_hist_counts=torch.empty(n, dtype=torch.int64, device="cuda"),
                         d_hist_len=torch.zeros(1, dtype=torch.int64, device="cuda")))
    gctx.count_batch(jobs)
    gctx.status()
    rng = np.random.default_rng(300)
    for q, c, j in zip(qs, sets, jobs):
        N = j["d_out_N"].cpu().numpy()
        idx = np.unique(np.concatenate([rng.integers(0, n, 12), [n - 1]]))
        assert np.array_equal(N[idx], oracle_mod.count_curves(q, 2, c[idx])), q
        L = int(j["d_hist_len"].item())
        k, cnt = _hist_np(N)
        assert L == len(k), q
        assert np.array_equal(j["d_hist_keys"][:L].cpu().numpy(), k), q
        assert np.array_equal(j["d_hist_counts"][:L].cpu().numpy().astype(np.uint64), cnt), q


def test_batch_g4_small_fields_sampled(gctx, oracle_mod, curvegen_mod):
    """g = 4 over q in {3, 5, 7, 9, 11, 13} in one launch: q = 3 fully
    enumerated (104 976 curves, all checked), the others 2^18 curves each,
    sampled."""
    import torch
    specs = [(3, curvegen_mod.enumerate_all(3, 4))]
    for q in (5, 7, 9, 11, 13):
        specs.append((q, curvegen_mod.sample(q, 4, 1 << 18, seed=curvegen_mod.BASE_SEED + 3 + q)))
    jobs = []
    for q, c in specs:
        n = len(c)
        jobs.append(dict(q=q, g=4, d_coeffs=torch.from_numpy(c).cuda(),
                         d_out_N=torch.empty((n, 4), dtype=torch.int32, device="cuda")))
    gctx.count_batch(jobs)
    gctx.status()
    rng = np.random.default_rng(15)
    for (q, c), j in zip(specs, jobs):
        N = j["d_out_N"].cpu().numpy()
        if q == 3:
            assert np.array_equal(N, oracle_mod.count_curves(3, 4, c))
        else:
            idx = np.unique(np.concatenate([rng.integers(0, len(c), 40), [len(c) - 1]]))
            assert np.array_equal(N[idx], oracle_mod.count_curves(q, 4, c[idx])), q


@pytest.mark.gpu
def test_valu_issue_rate_is_at_most_one_per_cu_clock(gctx):
    # the diagnostic issue-rate kernel: plain 32-bit instructions reach at most
    # one wave64 instruction per CU per clock (4 SIMDs x 16 lanes), 256 CUs at
    # no more than 2.4 GHz, and well above a quarter of it
    r = gctx.valu_issue_rate()
    assert 0.25 * 256 * 2.4e9 < r <= 1.05 * 256 * 2.4e9, r


@pytest.mark.gpu
def test_lds_gather_rate_is_below_the_bank_peak(gctx):
    from paper_1805_11991_amd import hwcount
    # the diagnostic gather kernel: a positive rate no faster than 32 u16 reads
    # per CU per clock (256 CUs, at most 2.4 GHz), and bad arguments rejected
    peak = 32 * 256 * 2.4e9
    for chains in (1, 4):
        r = gctx.lds_gather_rate(4392, chains)
        assert 0 < r <= peak * 1.05, r
    for entries, chains in ((10, 4), (1 << 20, 4), (4392, 3)):
        with pytest.raises(hwcount.HwcError):
            gctx.lds_gather_rate(entries, chains)
