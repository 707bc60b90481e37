"""Python binding of libhwcount.so (include/hwcount.h), same names.

Argument marshalling only: every step of the count runs in the library's HIP
kernels.  Device buffers are torch tensors (PyTorch supplies device memory and
streams); host calls take numpy arrays.  Importing this module does not need a
GPU, but it fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhwcount.so")

HWC_OK = 0
HWC_ERR_NOT_ODD_PRIME_POWER = -1
HWC_ERR_BAD_G = -2
HWC_ERR_FIELD_TOO_LARGE = -3
HWC_ERR_COEFF_RANGE = -4
HWC_ERR_DEGREE = -5
HWC_ERR_HIST_CAPACITY = -6
HWC_ERR_OOM_BUDGET = -7
HWC_ERR_DEVICE = -8
HWC_ERR_SINGULAR = -9
HWC_ERR_ARG = -10
HWC_ERR_NO_DEVICE = -11

HWC_FULL_SWEEP = 1
HWC_PLAIN = 2
HWC_VALIDATE = 4
HWC_NO_GRAPH = 8

HWC_OPT_SPLIT = 1
HWC_OPT_BLOCK = 2
HWC_OPT_WG_PER_CU = 3
HWC_OPT_DEVICE_TABLES = 4
HWC_OPT_WAVES_PER_SIMD = 5
HWC_OPT_SPLIT_MIN_M = 6
HWC_OPT_SHIFT = 7
HWC_OPT_MFMA = 8

#: every symbol the header declares
EXPORTS = ("hwc_ctx_create", "hwc_ctx_destroy", "hwc_last_error", "hwc_build_field", "hwc_field_info",
           "hwc_field_tables", "hwc_field_release", "hwc_count_curves", "hwc_count_curves_dev",
           "hwc_count_lambda_dev", "hwc_count_map", "hwc_count_single", "hwc_lds_gather_rate", "hwc_valu_issue_rate",
           "hwc_translate_dev", "hwc_count_batch", "hwc_ctx_status", "hwc_ctx_stats", "hwc_ctx_profile",
           "hwc_ctx_profile_read", "hwc_plan_info", "hwc_ctx_set_option", "hwc_ctx_set_plan_option",
           "hwc_ctx_reserve", "hwc_count_curves_dev_noalloc", "hwc_device_gather_rate")

#: bytes of the static scratch array of hwc_count_curves_dev_noalloc (per GPU)
HWC_NOALLOC_SCRATCH_BYTES = 64 << 20


class HwcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hwcount error {code}: {msg}")
        self.code = code


class hwc_field_desc(ctypes.Structure):
    _fields_ = [("p", ctypes.c_uint32), ("e", ctypes.c_uint32), ("k", ctypes.c_uint32), ("n", ctypes.c_uint32),
                ("q", ctypes.c_uint64), ("Q", ctypes.c_uint64), ("modulus", ctypes.c_uint32 * 41),
                ("qmodulus", ctypes.c_uint32 * 41), ("root_log", ctypes.c_uint32),
                ("nprim_orbits", ctypes.c_uint64), ("table_bytes", ctypes.c_uint64)]


class hwc_hist(ctypes.Structure):
    _fields_ = [("g", ctypes.c_uint32), ("capacity", ctypes.c_uint64), ("len", ctypes.c_uint64),
                ("keys", ctypes.c_void_p), ("counts", ctypes.c_void_p)]


class hwc_level_desc(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in ("M", "form", "nx", "weight", "msplit", "nt", "ns", "lds_bytes", "mfma")]


class hwc_job(ctypes.Structure):
    _fields_ = [("q", ctypes.c_uint32), ("g", ctypes.c_uint32), ("d_coeffs", ctypes.c_void_p),
                ("coeff_bytes", ctypes.c_int), ("n", ctypes.c_uint64), ("d_out_N", ctypes.c_void_p),
                ("d_hist_keys", ctypes.c_void_p), ("d_hist_counts", ctypes.c_void_p),
                ("hist_capacity", ctypes.c_uint64), ("d_hist_len", ctypes.c_void_p)]


_lib = None


def load():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1805_11991_amd.build`")
    # PyTorch ships its own HIP runtime, which its libraries find by a name that
    # differs from the library's dependency.  Loading torch first lets the
    # library bind to that same runtime (one runtime per process, so device
    # pointers and streams are shared); loading the library first would put a
    # second runtime into the process and leave torch without devices.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "hwc_ctx_create": (i32, [i32, u64, ctypes.POINTER(vp)]),
        "hwc_ctx_destroy": (None, [vp]),
        "hwc_last_error": (ctypes.c_char_p, [vp]),
        "hwc_build_field": (i32, [vp, u32, u32, u32, ctypes.POINTER(vp)]),
        "hwc_field_info": (i32, [vp, ctypes.POINTER(hwc_field_desc)]),
        "hwc_field_tables": (i32, [vp, vp, vp, vp, vp, vp]),
        "hwc_field_release": (None, [vp]),
        "hwc_count_curves": (i32, [vp, u32, u32, vp, u64, vp, ctypes.POINTER(hwc_hist), u32]),
        "hwc_count_curves_dev": (i32, [vp, u32, u32, vp, i32, u64, vp, vp, vp, u64, vp, u32, vp]),
        "hwc_count_curves_dev_noalloc": (i32, [vp, u32, u32, vp, i32, u64, vp, vp, vp, u64, vp, u32, vp]),
        "hwc_count_lambda_dev": (i32, [vp, u32, u32, vp, i32, u64, vp, vp, vp, vp, u64, vp, u32, vp]),
        "hwc_count_map": (i32, [vp, u32, u32, vp, vp, u64, ctypes.POINTER(u64), ctypes.POINTER(u64), u32]),
        "hwc_count_single": (i32, [vp, u32, u32, vp, u32, vp, vp, u32]),
        "hwc_lds_gather_rate": (i32, [vp, u32, u32, ctypes.POINTER(ctypes.c_double)]),
        "hwc_valu_issue_rate": (i32, [vp, ctypes.POINTER(ctypes.c_double)]),
        "hwc_device_gather_rate": (i32, [vp, u64, u32, ctypes.POINTER(ctypes.c_double)]),
        "hwc_translate_dev": (i32, [vp, u32, u32, vp, i32, u64, vp, vp]),
        "hwc_count_batch": (i32, [vp, ctypes.POINTER(hwc_job), ctypes.c_size_t, u32, vp]),
        "hwc_ctx_status": (i32, [vp, vp]),
        "hwc_ctx_stats": (i32, [vp, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u64),
                                ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u64)]),
        "hwc_ctx_reserve": (i32, [vp, u64, u32, vp]),
        "hwc_ctx_profile": (i32, [vp, i32]),
        "hwc_ctx_set_option": (i32, [vp, i32, ctypes.c_int64]),
        "hwc_ctx_set_plan_option": (i32, [vp, u32, u32, u32, i32, ctypes.c_int64]),
        "hwc_plan_info": (i32, [vp, u32, u32, u32, ctypes.POINTER(hwc_level_desc)]),
        "hwc_ctx_profile_read": (i32, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t) -> int | None:
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    return int(t.data_ptr())


class Field:
    def __init__(self, ctx: "Context", handle):
        self._ctx = ctx
        self._h = handle

    def info(self) -> hwc_field_desc:
        d = hwc_field_desc()
        self._ctx._check(load().hwc_field_info(self._h, ctypes.byref(d)))
        return d

    def tables(self) -> dict:
        d = self.info()
        M, Q, q = int(d.Q) - 1, int(d.Q), int(d.q)
        out = {"exp": np.zeros(M, np.uint32), "log": np.zeros(Q, np.uint32), "zech": np.zeros(M, np.uint32),
               "emb": np.zeros(q, np.uint32), "prim_reps": np.zeros(max(int(d.nprim_orbits), 1), np.uint32)}
        self._ctx._check(load().hwc_field_tables(self._h, *(a.ctypes.data for a in out.values())))
        out["prim_reps"] = out["prim_reps"][:int(d.nprim_orbits)]
        return out

    def release(self):
        if self._h:
            load().hwc_field_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Context:
    """hwc_ctx: device -1 gives a host-only context (fields only)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, autotune_db: str | None = "default",
                 mfma: bool = False):
        """autotune_db: path of a tuning database, "default" for the one of
        this architecture shipped with the package (if present), or None.
        mfma: opt in to the int8 matrix-product counting path for prime
        q <= 31 (HWC_OPT_MFMA) on every plan, tuned or not; the default is
        Zech-logarithm evaluation."""
        lib = load()
        h = ctypes.c_void_p()
        rc = lib.hwc_ctx_create(device, hbm_budget_bytes, ctypes.byref(h))
        if rc != HWC_OK:
            raise HwcError(rc, "hwc_ctx_create failed: " + (lib.hwc_last_error(None) or b"").decode())
        self._h = h
        self.device = device
        self.tuned_entries = 0
        if mfma:
            # before the tuning database: its per-plan entries start from the defaults
            self.set_option(HWC_OPT_MFMA, 1)
        if device >= 0 and autotune_db is not None:
            from . import autotune
            db = autotune.load_db(None if autotune_db == "default" else autotune_db)
            self.tuned_entries = autotune.apply_db(self, db)

    def _check(self, rc: int):
        if rc != HWC_OK:
            raise HwcError(rc, load().hwc_last_error(self._h).decode())

    def close(self):
        if self._h:
            load().hwc_ctx_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- fields
    def build_field(self, p: int, e: int, k: int) -> Field:
        h = ctypes.c_void_p()
        self._check(load().hwc_build_field(self._h, p, e, k, ctypes.byref(h)))
        return Field(self, h)

    # -- host-pointer count
    def count_curves(self, q: int, g: int, coeffs, flags: int = 0, want_N: bool = True,
                     hist_capacity: int | None = None):
        """Returns (N [n,g] int32 or None, (keys [len,g], counts [len]) or None)."""
        c = np.ascontiguousarray(np.asarray(coeffs), dtype=np.int16)
        if c.ndim != 2 or c.shape[1] != 2 * g + 3:
            raise ValueError(f"coeffs must be [n, {2 * g + 3}]")
        n = c.shape[0]
        N = np.zeros((n, g), np.int32) if want_N else None
        hist = None
        hk = hc = None
        if hist_capacity is not None:
            cap = max(int(hist_capacity), 0)
            hk = np.zeros((max(cap, 1), g), np.int32)
            hc = np.zeros(max(cap, 1), np.uint64)
            hist = hwc_hist(g, cap, 0, hk.ctypes.data, hc.ctypes.data)
        rc = load().hwc_count_curves(self._h, q, g, c.ctypes.data, n, N.ctypes.data if N is not None else None,
                                     ctypes.byref(hist) if hist is not None else None, flags)
        if rc == HWC_ERR_HIST_CAPACITY:
            raise HwcError(rc, f"histogram needs {hist.len} entries")
        self._check(rc)
        H = None
        if hist is not None:
            H = (hk[:hist.len].copy(), hc[:hist.len].copy())
        return N, H

    # -- device-pointer count (torch tensors)
    def count_curves_dev(self, q: int, g: int, d_coeffs, d_out_N, d_hist_keys=None, d_hist_counts=None,
                         d_hist_len=None, flags: int = 0, stream=None):
        cb = d_coeffs.element_size()
        n = d_coeffs.shape[0]
        cap = 0 if d_hist_keys is None else d_hist_keys.shape[0]
        s = None if stream is None else ctypes.c_void_p(int(stream.cuda_stream))
        self._check(load().hwc_count_curves_dev(self._h, q, g, _ptr(d_coeffs), cb, n, _ptr(d_out_N),
                                                _ptr(d_hist_keys), _ptr(d_hist_counts), cap, _ptr(d_hist_len),
                                                flags, s))

    def count_curves_dev_noalloc(self, q: int, g: int, d_coeffs, d_out_N, d_hist_keys=None, d_hist_counts=None,
                                 d_hist_len=None, flags: int = 0, stream=None):
        """hwc_count_curves_dev_noalloc: as count_curves_dev, allocating nothing
        (the plan of (q, g) must be resident; scratch is the GPU's static array)."""
        cb = d_coeffs.element_size()
        n = d_coeffs.shape[0]
        cap = 0 if d_hist_keys is None else d_hist_keys.shape[0]
        s = None if stream is None else ctypes.c_void_p(int(stream.cuda_stream))
        self._check(load().hwc_count_curves_dev_noalloc(self._h, q, g, _ptr(d_coeffs), cb, n, _ptr(d_out_N),
                                                        _ptr(d_hist_keys), _ptr(d_hist_counts), cap,
                                                        _ptr(d_hist_len), flags, s))

    def count_lambda_dev(self, q: int, g: int, d_coeffs, d_out_N, d_out_lambda, d_hist_keys=None,
                         d_hist_counts=None, d_hist_len=None, flags: int = 0, stream=None):
        """N and the factorization partition code of every row (torch tensors:
        d_out_lambda int32/uint32 [n]; histogram keys [cap, g+1])."""
        cap = 0 if d_hist_keys is None else d_hist_keys.shape[0]
        s = None if stream is None else ctypes.c_void_p(int(stream.cuda_stream))
        self._check(load().hwc_count_lambda_dev(self._h, q, g, _ptr(d_coeffs), d_coeffs.element_size(),
                                                d_coeffs.shape[0], _ptr(d_out_N), _ptr(d_out_lambda),
                                                _ptr(d_hist_keys), _ptr(d_hist_counts), cap, _ptr(d_hist_len),
                                                flags, s))

    def count_map(self, q: int, g: int, flags: int = 0, capacity: int = 1 << 20):
        """The map N_{g,q} of eq. (1.2) by Algorithm 1.  Returns (keys [len, g+1]
        int32: a_1..a_g and the factorization code, counts [len] uint64, number
        of representatives evaluated)."""
        while True:
            keys = np.zeros((max(capacity, 1), g + 1), np.int32)
            counts = np.zeros(max(capacity, 1), np.uint64)
            n = ctypes.c_uint64()
            reps = ctypes.c_uint64()
            rc = load().hwc_count_map(self._h, q, g, keys.ctypes.data, counts.ctypes.data, capacity,
                                      ctypes.byref(n), ctypes.byref(reps), flags)
            if rc == HWC_ERR_HIST_CAPACITY and n.value > capacity:
                capacity = int(n.value)
                continue
            self._check(rc)
            return keys[:n.value].copy(), counts[:n.value].copy(), int(reps.value)

    def count_single(self, q: int, g: int, coeffs, kmax: int, flags: int = 0):
        """One curve (codes [2g+3]) over F_{q^k}, k = 1..kmax, lane per x.
        Returns (N int64 [kmax], timings dict in ms: tables, upload, kernels)."""
        c = np.ascontiguousarray(np.asarray(coeffs), dtype=np.int16).reshape(-1)
        if c.shape[0] != 2 * g + 3:
            raise ValueError(f"coeffs must have {2 * g + 3} codes")
        out = np.zeros(kmax, np.int64)
        t = np.zeros(3, np.float64)
        self._check(load().hwc_count_single(self._h, q, g, c.ctypes.data, kmax, out.ctypes.data, t.ctypes.data,
                                            flags))
        return out, {"tables_ms": float(t[0]), "upload_ms": float(t[1]), "kernel_ms": float(t[2])}

    def translate_dev(self, q: int, g: int, d_coeffs, d_out, stream=None):
        """The rows the counting calls evaluate (dense translates), into d_out
        (torch tensor shaped and typed like d_coeffs)."""
        if d_out.shape != d_coeffs.shape or d_out.dtype != d_coeffs.dtype:
            raise ValueError("d_out must match d_coeffs in shape and dtype")
        s = None if stream is None else ctypes.c_void_p(int(stream.cuda_stream))
        self._check(load().hwc_translate_dev(self._h, q, g, _ptr(d_coeffs), d_coeffs.element_size(),
                                             d_coeffs.shape[0], _ptr(d_out), s))

    def lds_gather_rate(self, table_entries: int, chains: int = 4) -> float:
        """Measured dependent random u16 LDS gathers per second (diagnostic)."""
        r = ctypes.c_double()
        self._check(load().hwc_lds_gather_rate(self._h, table_entries, chains, ctypes.byref(r)))
        return r.value

    def valu_issue_rate(self) -> float:
        """Measured wave64 issue rate of plain 32-bit vector instructions, per second (diagnostic)."""
        r = ctypes.c_double()
        self._check(load().hwc_valu_issue_rate(self._h, ctypes.byref(r)))
        return r.value

    def device_gather_rate(self, table_entries: int, chains: int = 4) -> float:
        """Measured dependent random u32 gathers per second from a device-memory table (diagnostic)."""
        r = ctypes.c_double()
        self._check(load().hwc_device_gather_rate(self._h, table_entries, chains, ctypes.byref(r)))
        return r.value

    def count_batch(self, jobs: list[dict], flags: int = 0, stream=None):
        arr = (hwc_job * max(len(jobs), 1))()
        for i, j in enumerate(jobs):
            hk = j.get("d_hist_keys")
            arr[i] = hwc_job(j["q"], j["g"], _ptr(j["d_coeffs"]), j["d_coeffs"].element_size(),
                             j["d_coeffs"].shape[0], _ptr(j["d_out_N"]), _ptr(hk), _ptr(j.get("d_hist_counts")),
                             0 if hk is None else hk.shape[0], _ptr(j.get("d_hist_len")))
        s = None if stream is None else ctypes.c_void_p(int(stream.cuda_stream))
        self._check(load().hwc_count_batch(self._h, arr, len(jobs), flags, s))

    def status(self, stream=None):
        s = None if stream is None else ctypes.c_void_p(int(stream.cuda_stream))
        self._check(load().hwc_ctx_status(self._h, s))

    def profile(self, enable: bool = True):
        self._check(load().hwc_ctx_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        t = [ctypes.c_double() for _ in range(3)]
        n = ctypes.c_uint64()
        self._check(load().hwc_ctx_profile_read(self._h, *(ctypes.byref(x) for x in t), ctypes.byref(n)))
        return {"prep_ms": t[0].value, "count_ms": t[1].value, "hist_ms": t[2].value, "calls": n.value}

    def set_option(self, opt: int, value: int):
        self._check(load().hwc_ctx_set_option(self._h, opt, value))

    def set_plan_option(self, q: int, g: int, opt: int, value: int, flags: int = 0):
        self._check(load().hwc_ctx_set_plan_option(self._h, q, g, flags, opt, value))

    def plan_info(self, q: int, g: int, flags: int = 0) -> list[dict]:
        arr = (hwc_level_desc * g)()
        self._check(load().hwc_plan_info(self._h, q, g, flags, arr))
        return [{f: getattr(a, f) for f, _ in hwc_level_desc._fields_} for a in arr]

    def stats(self) -> dict:
        v = [ctypes.c_uint64() for _ in range(6)]
        self._check(load().hwc_ctx_stats(self._h, *(ctypes.byref(x) for x in v)))
        return dict(zip(("plans_resident", "table_bytes", "cache_hits", "cache_misses", "evictions",
                         "pending_free_bytes"), (x.value for x in v)))

    def reserve(self, max_curves: int, max_jobs: int = 64, stream=None):
        """Preallocate the scratch of the calls on `stream` (hwc_ctx_reserve)."""
        s = None if stream is None else ctypes.c_void_p(int(stream.cuda_stream))
        self._check(load().hwc_ctx_reserve(self._h, max_curves, max_jobs, s))


LAMBDA_SHIFT = (0, 4, 7, 9, 11, 13, 14, 15, 16, 17)
LAMBDA_WIDTH = (4, 3, 2, 2, 2, 1, 1, 1, 1, 1)
LAMBDA_INVALID = 0xFFFFFFFF


def lambda_multiplicities(codes, g: int):
    """Decode factorization codes into multiplicities: int array [n, 2g+2],
    column j-1 = number of parts equal to j."""
    c = np.asarray(codes).astype(np.uint64) & 0xFFFFFFFF
    out = np.zeros((c.shape[0], 2 * g + 2), dtype=np.int64)
    for j in range(1, 2 * g + 3):
        out[:, j - 1] = (c >> LAMBDA_SHIFT[j - 1]) & ((1 << LAMBDA_WIDTH[j - 1]) - 1)
    return out


def lambda_code(mults) -> int:
    """Code of one partition given by its multiplicities (index j-1 = part j)."""
    v = 0
    for j, m in enumerate(mults, start=1):
        if m:
            assert m < (1 << LAMBDA_WIDTH[j - 1])
            v |= int(m) << LAMBDA_SHIFT[j - 1]
    return v
