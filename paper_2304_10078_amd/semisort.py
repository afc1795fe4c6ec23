"""Python binding of libsemisort_hip.so (C-ABI in include/semisort.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Arrays are torch tensors on the GPU; uint64 keys and values travel
as int64 tensors holding the same bit patterns (uint32 values as int32).
Work is issued on torch's current HIP stream.  If the library is not built,
importing the functions raises immediately -- there is no fallback.
"""
import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsemisort_hip.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "semisort.h")

SS_OK, SS_EINVAL, SS_ENOMEM, SS_EHIP, SS_EDEVICE = 0, -1, -2, -3, -4
HASH_MIX64, HASH_IDENTITY = 0, 1
HEAVY_MAX = 512
LIGHT_BITS_MAX = 10

_STATUS = {SS_EINVAL: "SS_EINVAL", SS_ENOMEM: "SS_ENOMEM", SS_EHIP: "SS_EHIP", SS_EDEVICE: "SS_EDEVICE"}


class SemisortError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class ss_params(ctypes.Structure):
    _fields_ = [
        ("n_light_log2", ctypes.c_uint32),
        ("base_case", ctypes.c_uint32),
        ("sample_mult", ctypes.c_uint32),
        ("tile_min", ctypes.c_uint32),
        ("tile_max", ctypes.c_uint32),
        ("hash_mode", ctypes.c_uint32),
        ("heavy_min", ctypes.c_uint32),
        ("temp_records", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
    ]


_lib = None


def declared_symbols():
    """Entry points declared in include/semisort.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:ss_status|const char\*|double)\s+(ss_\w+)\s*\(", txt, re.M)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(the GPU path has no fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        P = ctypes.POINTER(ss_params)
        L.ss_default_params.argtypes = [P]
        L.ss_create.argtypes = [i32, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.ss_destroy.argtypes = [vp]
        L.ss_set_stream.argtypes = [vp, vp]
        L.ss_last_error.argtypes = [vp]
        L.ss_last_error.restype = ctypes.c_char_p
        L.ss_sync.argtypes = [vp]
        L.ss_workspace_held.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.ss_workspace_bytes.argtypes = [i32, u64, u32, P, ctypes.POINTER(ctypes.c_size_t)]
        L.ss_collect_reduce_async.argtypes = [vp, vp, vp, u64, i32, i32, vp, vp, vp, P]
        L.ss_histogram_async.argtypes = [vp, vp, u64, i32, vp, vp, vp, P]
        L.ss_batch.argtypes = [vp, vp, u64, P]
        L.ss_profile_enable.argtypes = [vp, i32]
        L.ss_set_option.argtypes = [vp, i32, ctypes.c_int64]
        L.ss_profile_read.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64),
                                      ctypes.POINTER(u64)]
        L.ss_semisort_equal.argtypes = [vp, vp, vp, u32, u64, vp, vp, P]
        L.ss_semisort_equal_batch.argtypes = [vp, vp, vp, u32, vp, u64, vp, vp, P]
        L.ss_semisort_less.argtypes = [vp, vp, vp, u32, u64, vp, vp, P]
        L.ss_semisort_equal_keys.argtypes = [vp, vp, u32, vp, u32, u64, vp, vp, P]
        L.ss_semisort_less_keys.argtypes = [vp, vp, u32, vp, u32, u64, vp, vp, P]
        L.ss_monoid_compile.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(vp)]
        L.ss_semisort_equal_batch_tuned.argtypes = [vp, vp, vp, u32, vp, u64, vp, vp, P, ctypes.POINTER(ctypes.c_int)]
        L.ss_autotune_cache.argtypes = [vp, ctypes.c_int, ctypes.POINTER(u64)]
        L.ss_monoid_destroy.argtypes = [vp]
        L.ss_collect_reduce_user.argtypes = [vp, vp, vp, vp, u32, u64, ctypes.c_int, vp, vp, ctypes.POINTER(u64), P]
        L.ss_semisort_less_batch.argtypes = [vp, vp, vp, u32, vp, u64, vp, vp, P]
        L.ss_partition_equal.argtypes = [vp, vp, vp, u32, u64, vp, vp, vp, vp, ctypes.POINTER(u32), P]
        L.ss_collect_reduce.argtypes = [vp, vp, vp, u64, vp, vp, ctypes.POINTER(u64), P]
        L.ss_autotune_equal_batch.argtypes = [vp, vp, vp, u32, vp, u64, vp, vp, u32, P,
                                              ctypes.POINTER(ctypes.c_double)]
        L.ss_histogram.argtypes = [vp, vp, u64, vp, vp, ctypes.POINTER(u64), P]
        L.ss_semisort_equal_batch_capturable.argtypes = [vp, vp, vp, u32, vp, u64, u64, vp, vp, u32, P]
        L.ss_semisort_equal_batch_noalloc.argtypes = L.ss_semisort_equal_batch_capturable.argtypes
        L.ss_collect_reduce_monoid.argtypes = [vp, vp, vp, u64, i32, i32, vp, vp, ctypes.POINTER(u64), P]
        L.ss_transpose_csr.argtypes = [vp, u64, u64, vp, vp, vp, vp, P]
        L.ss_collect_reduce_ordered.argtypes = L.ss_collect_reduce.argtypes
        L.ss_histogram_ordered.argtypes = L.ss_histogram.argtypes
        for name in declared_symbols():
            if name != "ss_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def default_params(**kw):
    p = ss_params()
    lib().ss_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k == "hash_mode" and isinstance(v, str):
            v = {"mix64": HASH_MIX64, "identity": HASH_IDENTITY}[v]
        setattr(p, k, v)
    return p


class Context:
    """One library context (ss_ctx) on a device; reuses its workspace across calls."""

    def __init__(self, device=0, workspace_cap=0):
        import torch
        self.device = device
        h = ctypes.c_void_p()
        st = lib().ss_create(device, ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream),
                             int(workspace_cap), ctypes.byref(h))
        if st != SS_OK:
            raise SemisortError(st, "ss_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().ss_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind_stream(self):
        import torch
        lib().ss_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def check(self, st):
        if st != SS_OK:
            raise SemisortError(st, lib().ss_last_error(self.h).decode())

    PROF_KINDS = ("sample", "count", "scan", "distribute", "plan", "finish", "compact", "fill")
    OPT_DIST_VARIANT = 1
    OPT_DEEP_SAMPLE_DIV = 2
    OPT_NL_TARGET = 3
    OPT_TILE0 = 4
    OPT_TILE_DEEP = 5
    OPT_FOLD_ROUND = 6

    def sync(self):
        """Wait for the context's stream; raises SemisortError for a device
        condition raised by earlier calls (see ss_sync)."""
        self.check(lib().ss_sync(self.h))

    def set_option(self, option, value):
        self.check(lib().ss_set_option(self.h, int(option), int(value)))

    def profile_enable(self, on=True):
        self.check(lib().ss_profile_enable(self.h, 1 if on else 0))

    def profile_read(self):
        """{pass: (total_ms, launches, units)} accumulated since profile_enable."""
        out = {}
        for k, name in enumerate(self.PROF_KINDS):
            ms = ctypes.c_double()
            la = ctypes.c_uint64()
            un = ctypes.c_uint64()
            self.check(lib().ss_profile_read(self.h, k, ctypes.byref(ms), ctypes.byref(la), ctypes.byref(un)))
            out[name] = (ms.value, la.value, un.value)
        return out

    def workspace_held(self):
        """ss_workspace_held: bytes of workspace the context holds now."""
        b = ctypes.c_size_t()
        self.check(lib().ss_workspace_held(self.h, ctypes.byref(b)))
        return b.value


def workspace_bound(op, n, val_bytes=8, params=None):
    """ss_workspace_bytes: upper bound of the workspace one call of `op` on n
    records makes a new context hold (a planning query; no device needed)."""
    b = ctypes.c_size_t()
    st = lib().ss_workspace_bytes(int(op), int(n), int(val_bytes),
                                  ctypes.byref(params) if params is not None else None, ctypes.byref(b))
    if st != SS_OK:
        raise SemisortError(st, "ss_workspace_bytes rejected its arguments")
    return b.value


_ctx = {}


def context(device=0):
    if device not in _ctx:
        _ctx[device] = Context(device)
    return _ctx[device]


def sync(device=0):
    """ss_sync on the device's default context."""
    context(device).sync()


def _check_kv(keys, vals, allow_k32=False):
    """Value width of a (keys, vals) pair of device tensors.  Keys: int64
    (uint64 bits), or with allow_k32 also int32 (uint32 bits) and an (n, 2)
    int64 tensor of 128-bit keys as (low, high) words."""
    import torch
    if not (keys.is_cuda and vals.is_cuda):
        raise ValueError("keys and vals must be device tensors")
    wide = allow_k32 and keys.dim() == 2 and keys.shape[-1] == 2 and keys.dtype == torch.int64
    kd = (torch.int64, torch.int32) if allow_k32 else (torch.int64,)
    if keys.dtype not in kd or vals.dtype not in (torch.int64, torch.int32):
        raise ValueError("keys must be int64 (uint64 bits)" +
                         (", int32 (uint32 bits) or (n, 2) int64 (128-bit)" if allow_k32 else "") +
                         ", vals int64 or int32 (uint bits)")
    if (keys.dim() != (2 if wide else 1) or vals.dim() != 1 or vals.shape[0] != keys.shape[0]
            or not keys.is_contiguous() or not vals.is_contiguous()):
        raise ValueError("keys and vals must be contiguous tensors of equal length (1-D, or (n, 2) keys)")
    return vals.element_size()


def _check_out(name, out, like):
    """An output tensor must hold at least what the input it stands for holds
    (device, dtype, row shape, at least as many rows, contiguous): the library
    writes up to as many bytes as the input has."""
    if (not out.is_cuda or out.device != like.device or out.dtype != like.dtype or out.dim() != like.dim()
            or out.shape[1:] != like.shape[1:] or out.shape[0] < like.shape[0] or not out.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous device tensor of at least the input's size "
                         f"({like.dtype}, {tuple(like.shape)})")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _semisort(less, keys, vals, keys_out, vals_out, params, ctx):
    import torch
    vb = _check_kv(keys, vals, allow_k32=True)
    n = keys.shape[0]
    kb = keys.element_size() * (2 if keys.dim() == 2 else 1)  # 4 or 16: ss_semisort_*_keys
    ctx = ctx or context(keys.device.index or 0)
    ctx._bind_stream()
    if keys_out is None:
        keys_out = torch.empty_like(keys)
    if vals_out is None:
        vals_out = torch.empty_like(vals)
    _check_out("keys_out", keys_out, keys)
    _check_out("vals_out", vals_out, vals)
    pp = ctypes.byref(params) if params is not None else None
    if kb != 8:
        fn = lib().ss_semisort_less_keys if less else lib().ss_semisort_equal_keys
        ctx.check(fn(ctx.h, _ptr(keys), kb, _ptr(vals), vb, n, _ptr(keys_out), _ptr(vals_out), pp))
    else:
        fn = lib().ss_semisort_less if less else lib().ss_semisort_equal
        ctx.check(fn(ctx.h, _ptr(keys), _ptr(vals), vb, n, _ptr(keys_out), _ptr(vals_out), pp))
    return keys_out, vals_out


def semisort_equal(keys, vals, keys_out=None, vals_out=None, params=None, ctx=None):
    """ss_semisort_equal: equal keys contiguous, stable.  Returns (keys_out, vals_out).
    keys: int64 (uint64 bits), int32 (uint32 bits) or (n, 2) int64 (128-bit keys
    as low, high words): the last two through ss_semisort_equal_keys."""
    return _semisort(False, keys, vals, keys_out, vals_out, params, ctx)


def semisort_less(keys, vals, keys_out=None, vals_out=None, params=None, ctx=None):
    """ss_semisort_less: ascending keys, stable.  Returns (keys_out, vals_out).
    keys: int64 (uint64 bits) or int32 (uint32 bits: ss_semisort_less_keys)."""
    return _semisort(True, keys, vals, keys_out, vals_out, params, ctx)


def semisort_less_batch(keys, vals, seg_offsets, keys_out=None, vals_out=None, params=None, ctx=None):
    """ss_semisort_less_batch: independent instances packed back to back."""
    import numpy as np
    import torch
    vb = _check_kv(keys, vals)
    offs = np.ascontiguousarray(np.asarray(seg_offsets, dtype=np.uint64))
    ctx = ctx or context(keys.device.index or 0)
    ctx._bind_stream()
    if keys_out is None:
        keys_out = torch.empty_like(keys)
    if vals_out is None:
        vals_out = torch.empty_like(vals)
    _check_out("keys_out", keys_out, keys)
    _check_out("vals_out", vals_out, vals)
    ctx.check(lib().ss_semisort_less_batch(ctx.h, _ptr(keys), _ptr(vals), vb, ctypes.c_void_p(offs.ctypes.data),
                                           offs.size - 1, _ptr(keys_out), _ptr(vals_out),
                                           ctypes.byref(params) if params is not None else None))
    return keys_out, vals_out


def semisort_equal_batch(keys, vals, seg_offsets, keys_out=None, vals_out=None, params=None, ctx=None):
    """ss_semisort_equal_batch: independent instances packed back to back.
    seg_offsets: host sequence of nseg+1 boundaries."""
    import numpy as np
    import torch
    vb = _check_kv(keys, vals)
    offs = np.ascontiguousarray(np.asarray(seg_offsets, dtype=np.uint64))
    ctx = ctx or context(keys.device.index or 0)
    ctx._bind_stream()
    if keys_out is None:
        keys_out = torch.empty_like(keys)
    if vals_out is None:
        vals_out = torch.empty_like(vals)
    _check_out("keys_out", keys_out, keys)
    _check_out("vals_out", vals_out, vals)
    ctx.check(lib().ss_semisort_equal_batch(ctx.h, _ptr(keys), _ptr(vals), vb,
                                            ctypes.c_void_p(offs.ctypes.data), offs.size - 1, _ptr(keys_out),
                                            _ptr(vals_out), ctypes.byref(params) if params is not None else None))
    return keys_out, vals_out


def semisort_equal_batch_capturable(keys, vals, seg_offsets, keys_out=None, vals_out=None, max_levels=4,
                                    params=None, ctx=None):
    """ss_semisort_equal_batch_capturable: the batch sized on the device, so
    the call can be recorded into a graph (torch.cuda.graph) and replayed.
    seg_offsets: int64 DEVICE tensor of nseg+1 boundaries, the last = len(keys).
    Under capture, pass keys_out / vals_out (allocated before capture) and make
    one uncaptured call with the same sizes first, so the workspace is sized.
    max_levels=4: with the default n_light_log2 every input below 2^31 records
    needs at most two levels plus the rare third for keys that escape the
    sample; more levels left unfinished raise SemisortError at sync."""
    import torch
    vb = _check_kv(keys, vals)
    _check_keys(seg_offsets, "seg_offsets")
    if seg_offsets.numel() < 1:
        raise ValueError("seg_offsets needs nseg + 1 entries")
    ctx = ctx or context(keys.device.index or 0)
    ctx._bind_stream()
    if keys_out is None:
        keys_out = torch.empty_like(keys)
    if vals_out is None:
        vals_out = torch.empty_like(vals)
    _check_out("keys_out", keys_out, keys)
    _check_out("vals_out", vals_out, vals)
    ctx.check(lib().ss_semisort_equal_batch_capturable(
        ctx.h, _ptr(keys), _ptr(vals), vb, _ptr(seg_offsets), seg_offsets.numel() - 1, keys.numel(),
        _ptr(keys_out), _ptr(vals_out), max_levels, ctypes.byref(params) if params is not None else None))
    return keys_out, vals_out


def semisort_equal_batch_noalloc(keys, vals, seg_offsets, keys_out, vals_out, max_levels=4, params=None,
                                 ctx=None):
    """ss_semisort_equal_batch_noalloc: ss_semisort_equal_batch_capturable
    with its workspace in the library's static scratch array, so the call
    allocates nothing.  The outputs are passed in (this function allocates
    nothing either); seg_offsets is an int64 DEVICE tensor of nseg+1
    boundaries, the last = len(keys).  Calls on one device must not overlap."""
    vb = _check_kv(keys, vals)
    _check_keys(seg_offsets, "seg_offsets")
    if seg_offsets.numel() < 1:
        raise ValueError("seg_offsets needs nseg + 1 entries")
    if keys_out.shape != keys.shape or vals_out.shape != vals.shape or vals_out.dtype != vals.dtype:
        raise ValueError("outputs must match the inputs' shapes and value type")
    ctx = ctx or context(keys.device.index or 0)
    ctx._bind_stream()
    ctx.check(lib().ss_semisort_equal_batch_noalloc(
        ctx.h, _ptr(keys), _ptr(vals), vb, _ptr(seg_offsets), seg_offsets.numel() - 1, keys.numel(),
        _ptr(keys_out), _ptr(vals_out), max_levels, ctypes.byref(params) if params is not None else None))
    return keys_out, vals_out


def partition_equal(keys, vals, params=None, ctx=None):
    """ss_partition_equal: one level of Steps 1-2.  Returns (T_keys, T_vals, offsets, heavy_hashes)."""
    import torch
    vb = _check_kv(keys, vals)
    ctx = ctx or context(keys.device.index or 0)
    ctx._bind_stream()
    if params is None:
        params = default_params()
    tk = torch.empty_like(keys)
    tv = torch.empty_like(vals)
    nb_cap = (1 << params.n_light_log2) + HEAVY_MAX + 1
    off = torch.zeros(nb_cap, dtype=torch.int64, device=keys.device)
    hv = torch.zeros(HEAVY_MAX, dtype=torch.int64, device=keys.device)
    nh = ctypes.c_uint32()
    ctx.check(lib().ss_partition_equal(ctx.h, _ptr(keys), _ptr(vals), vb, keys.numel(), _ptr(tk), _ptr(tv),
                                       _ptr(off), _ptr(hv), ctypes.byref(nh), ctypes.byref(params)))
    nb = (1 << params.n_light_log2) + nh.value
    return tk, tv, off[:nb + 1], hv[:nh.value]


def _check_keys(keys, name="keys"):
    import torch
    if not keys.is_cuda or keys.dtype != torch.int64 or keys.dim() != 1 or not keys.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 1-D int64 device tensor (uint64 bits)")


MONOIDS = {"sum": 0, "min": 1, "max": 2, "xor": 3, "first": 4, "last": 5, "affine": 6}


class Monoid:
    """A caller's monoid compiled for one device (ss_monoid_compile).  `source`
    defines ss_t, ss_identity(), ss_map(ss_u64 value) and ss_combine(a, b)
    (associative, a first in input order) as __device__ functions."""

    def __init__(self, source, ctx=None, device=0):
        ctx = ctx or context(device)
        h = ctypes.c_void_p()
        ctx.check(lib().ss_monoid_compile(ctx.h, source.encode(), ctypes.byref(h)))
        self.h = h
        self.device = ctx.device

    def close(self):
        if getattr(self, "h", None):
            lib().ss_monoid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def collect_reduce_user(keys, vals, monoid, ordered=False, params=None, ctx=None, out_keys=None, out_vals=None):
    """ss_collect_reduce_user: (unique keys, fold of ss_map(value) over each
    key's records in input order with the monoid's ss_combine); vals int64 or
    int32 (uint bits).  Each result holds the element's bytes zero-extended to
    8.  Returns views of length m of the two output tensors (capacity n each)."""
    import torch
    _check_keys(keys)
    if not vals.is_cuda or vals.dtype not in (torch.int64, torch.int32) or vals.shape != keys.shape \
            or not vals.is_contiguous():
        raise ValueError("vals must be a contiguous int64 or int32 device tensor as long as keys")
    ctx = ctx or context(keys.device.index or 0)
    ctx._bind_stream()
    if out_keys is None:
        out_keys = torch.empty_like(keys)
    if out_vals is None:
        out_vals = torch.empty_like(keys)
    _check_out("out_keys", out_keys, keys)
    _check_out("out_vals", out_vals, keys)
    m = ctypes.c_uint64()
    ctx.check(lib().ss_collect_reduce_user(ctx.h, monoid.h, _ptr(keys), _ptr(vals), vals.element_size(),
                                           keys.numel(), int(bool(ordered)), _ptr(out_keys), _ptr(out_vals),
                                           ctypes.byref(m), ctypes.byref(params) if params is not None else None))
    return out_keys[:m.value], out_vals[:m.value]


def collect_reduce(keys, vals, params=None, ctx=None, out_keys=None, out_sums=None, ordered=False, op="sum"):
    """ss_collect_reduce: (unique keys, wrapping uint64 sums of their values);
    ss_collect_reduce_ordered with ordered=True (keys ascending as uint64);
    ss_collect_reduce_monoid for op in "min", "max", "xor", "first", "last"
    (uint64 values; first / last: the key's first / last record in input order).

    Returns views of length m of the two output tensors (capacity n each)."""
    import torch
    _check_keys(keys)
    _check_keys(vals, "vals")
    if vals.shape != keys.shape:
        raise ValueError("keys and vals must have equal length")
    ctx = ctx or context(keys.device.index or 0)
    ctx._bind_stream()
    if out_keys is None:
        out_keys = torch.empty_like(keys)
    if out_sums is None:
        out_sums = torch.empty_like(keys)
    _check_out("out_keys", out_keys, keys)
    _check_out("out_sums", out_sums, keys)
    m = ctypes.c_uint64()
    pp = ctypes.byref(params) if params is not None else None
    if op != "sum":
        ctx.check(lib().ss_collect_reduce_monoid(ctx.h, _ptr(keys), _ptr(vals), keys.numel(), MONOIDS[op],
                                                 int(bool(ordered)), _ptr(out_keys), _ptr(out_sums),
                                                 ctypes.byref(m), pp))
    else:
        fn = lib().ss_collect_reduce_ordered if ordered else lib().ss_collect_reduce
        ctx.check(fn(ctx.h, _ptr(keys), _ptr(vals), keys.numel(), _ptr(out_keys), _ptr(out_sums),
                     ctypes.byref(m), pp))
    return out_keys[:m.value], out_sums[:m.value]


def histogram(keys, params=None, ctx=None, out_keys=None, out_counts=None, ordered=False):
    """ss_histogram: (unique keys, occurrence counts) as views of length m;
    ss_histogram_ordered with ordered=True (keys ascending as uint64)."""
    import torch
    _check_keys(keys)
    ctx = ctx or context(keys.device.index or 0)
    ctx._bind_stream()
    if out_keys is None:
        out_keys = torch.empty_like(keys)
    if out_counts is None:
        out_counts = torch.empty_like(keys)
    _check_out("out_keys", out_keys, keys)
    _check_out("out_counts", out_counts, keys)
    m = ctypes.c_uint64()
    fn = lib().ss_histogram_ordered if ordered else lib().ss_histogram
    ctx.check(fn(ctx.h, _ptr(keys), keys.numel(), _ptr(out_keys), _ptr(out_counts),
                 ctypes.byref(m), ctypes.byref(params) if params is not None else None))
    return out_keys[:m.value], out_counts[:m.value]


def collect_reduce_async(keys, vals, d_m, out_keys, out_vals, op="sum", ordered=False, params=None, ctx=None):
    """ss_collect_reduce_async: like collect_reduce, but m goes to d_m (an
    int64 device tensor of one entry) and the call does not wait for it.
    The outputs have capacity n; their first m entries hold the pairs."""
    _check_keys(keys)
    _check_keys(vals, "vals")
    _check_keys(d_m, "d_m")
    if vals.shape != keys.shape or d_m.numel() < 1:
        raise ValueError("vals must be as long as keys, and d_m hold one entry")
    _check_out("out_keys", out_keys, keys)
    _check_out("out_vals", out_vals, keys)
    ctx = ctx or context(keys.device.index or 0)
    ctx._bind_stream()
    ctx.check(lib().ss_collect_reduce_async(ctx.h, _ptr(keys), _ptr(vals), keys.numel(), MONOIDS[op],
                                            int(bool(ordered)), _ptr(out_keys), _ptr(out_vals), _ptr(d_m),
                                            ctypes.byref(params) if params is not None else None))


def histogram_async(keys, d_m, out_keys, out_counts, ordered=False, params=None, ctx=None):
    """ss_histogram_async: like histogram, with m to the device tensor d_m."""
    _check_keys(keys)
    _check_keys(d_m, "d_m")
    if d_m.numel() < 1:
        raise ValueError("d_m must hold one entry")
    _check_out("out_keys", out_keys, keys)
    _check_out("out_counts", out_counts, keys)
    ctx = ctx or context(keys.device.index or 0)
    ctx._bind_stream()
    ctx.check(lib().ss_histogram_async(ctx.h, _ptr(keys), keys.numel(), int(bool(ordered)), _ptr(out_keys),
                                       _ptr(out_counts), _ptr(d_m),
                                       ctypes.byref(params) if params is not None else None))


class ss_job(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_int32),
        ("val_bytes", ctypes.c_uint32),
        ("n", ctypes.c_uint64),
        ("keys", ctypes.c_void_p),
        ("vals", ctypes.c_void_p),
        ("out_a", ctypes.c_void_p),
        ("out_b", ctypes.c_void_p),
        ("d_m", ctypes.c_void_p),
    ]


def batch(jobs, params=None, ctx=None):
    """ss_batch over a list of (op, keys, vals, out_a, out_b, d_m) tuples of
    device tensors (vals None for the histogram, d_m None for semisort; d_m
    is an int64 tensor whose first entry receives m).  Returns after the
    work is enqueued."""
    arr = (ss_job * max(1, len(jobs)))()
    dev = 0
    for i, (op, k, v, oa, ob, dm) in enumerate(jobs):
        j = arr[i]
        j.op = int(op)
        j.val_bytes = v.element_size() if v is not None else 8
        j.n = k.numel()
        j.keys = k.data_ptr() if k.numel() else None
        j.vals = v.data_ptr() if v is not None and v.numel() else None
        j.out_a = oa.data_ptr() if oa.numel() else None
        j.out_b = ob.data_ptr() if ob.numel() else None
        j.d_m = dm.data_ptr() if dm is not None else None
        dev = k.device.index or 0
    ctx = ctx or context(dev)
    ctx._bind_stream()
    ctx.check(lib().ss_batch(ctx.h, arr, len(jobs), ctypes.byref(params) if params is not None else None))


def transpose_csr(offsets, cols, params=None, ctx=None, out_offsets=None, out_cols=None):
    """ss_transpose_csr: the transpose of a CSR graph.  offsets: int64 device
    tensor of nv + 1 entries; cols: int32 device tensor of targets (uint32
    bits).  Returns (out_offsets, out_cols) of the same shapes."""
    import torch
    _check_keys(offsets, "offsets")
    if not cols.is_cuda or cols.dtype != torch.int32 or cols.dim() != 1 or not cols.is_contiguous():
        raise ValueError("cols must be a contiguous 1-D int32 device tensor (uint32 bits)")
    ctx = ctx or context(offsets.device.index or 0)
    ctx._bind_stream()
    if out_offsets is None:
        out_offsets = torch.empty_like(offsets)
    if out_cols is None:
        out_cols = torch.empty_like(cols)
    ctx.check(lib().ss_transpose_csr(ctx.h, offsets.numel() - 1, cols.numel(), _ptr(offsets), _ptr(cols),
                                     _ptr(out_offsets), _ptr(out_cols),
                                     ctypes.byref(params) if params is not None else None))
    return out_offsets, out_cols


def semisort_equal_batch_tuned(keys, vals, seg_offsets, keys_out=None, vals_out=None, ctx=None):
    """ss_semisort_equal_batch_tuned: the batch semisorted with the parameters
    the context tuned for its class (tuning them on the first batch of a
    class).  Returns (keys_out, vals_out, parameters used, tuned now)."""
    import numpy as np
    import torch
    vb = _check_kv(keys, vals)
    ctx = ctx or context(keys.device.index or 0)
    ctx._bind_stream()
    offs = np.ascontiguousarray(np.asarray(seg_offsets, dtype=np.uint64))
    if keys_out is None:
        keys_out = torch.empty_like(keys)
    if vals_out is None:
        vals_out = torch.empty_like(vals)
    _check_out("keys_out", keys_out, keys)
    _check_out("vals_out", vals_out, vals)
    used = ss_params()
    now = ctypes.c_int()
    ctx.check(lib().ss_semisort_equal_batch_tuned(ctx.h, _ptr(keys), _ptr(vals), vb,
                                                  offs.ctypes.data_as(ctypes.c_void_p), offs.size - 1,
                                                  _ptr(keys_out), _ptr(vals_out), ctypes.byref(used),
                                                  ctypes.byref(now)))
    return keys_out, vals_out, used, bool(now.value)


def autotune_cache(clear=False, ctx=None, device=0):
    """ss_autotune_cache: number of batch classes with tuned parameters (after
    forgetting them all with clear=True)."""
    ctx = ctx or context(device)
    e = ctypes.c_uint64()
    ctx.check(lib().ss_autotune_cache(ctx.h, int(bool(clear)), ctypes.byref(e)))
    return e.value


def autotune_equal_batch(keys, vals, seg_offsets, keys_out=None, vals_out=None, reps=2, ctx=None):
    """ss_autotune_equal_batch: (best ss_params, ms per run with them).  The
    outputs hold the batch's semisort afterwards."""
    import numpy as np
    import torch
    vb = _check_kv(keys, vals)
    ctx = ctx or context(keys.device.index or 0)
    ctx._bind_stream()
    offs = np.ascontiguousarray(np.asarray(seg_offsets, dtype=np.uint64))
    if keys_out is None:
        keys_out = torch.empty_like(keys)
    if vals_out is None:
        vals_out = torch.empty_like(vals)
    _check_out("keys_out", keys_out, keys)
    _check_out("vals_out", vals_out, vals)
    best = ss_params()
    ms = ctypes.c_double()
    ctx.check(lib().ss_autotune_equal_batch(ctx.h, _ptr(keys), _ptr(vals), vb, offs.ctypes.data_as(ctypes.c_void_p),
                                            offs.size - 1, _ptr(keys_out), _ptr(vals_out), int(reps),
                                            ctypes.byref(best), ctypes.byref(ms)))
    return best, ms.value


# ---------------------------------------------------------------- serving

OP_SEMISORT_EQUAL, OP_SEMISORT_LESS, OP_HISTOGRAM, OP_COLLECT_REDUCE = 0, 1, 2, 3


class ss_request(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_int32),
        ("val_bytes", ctypes.c_uint32),
        ("n", ctypes.c_uint64),
        ("keys", ctypes.c_void_p),
        ("vals", ctypes.c_void_p),
        ("out_a", ctypes.c_void_p),
        ("out_b", ctypes.c_void_p),
    ]


class ss_server_config(ctypes.Structure):
    _fields_ = [
        ("lanes", ctypes.c_uint32),
        ("pack_max_records", ctypes.c_uint32),
        ("batch_records", ctypes.c_uint64),
        ("hbm_budget", ctypes.c_uint64),
        ("params", ss_params),
    ]


def _bind_server(L):
    vp, u64 = ctypes.c_void_p, ctypes.c_uint64
    L.ss_server_default_config.argtypes = [ctypes.POINTER(ss_server_config)]
    L.ss_server_create.argtypes = [ctypes.c_int, ctypes.POINTER(ss_server_config), ctypes.POINTER(vp)]
    L.ss_server_now.argtypes = [vp]
    L.ss_server_now.restype = ctypes.c_double
    L.ss_server_submit.argtypes = [vp, ctypes.POINTER(ss_request), ctypes.c_double, ctypes.POINTER(u64)]
    L.ss_server_poll.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64)]
    L.ss_server_drain.argtypes = [vp]
    L.ss_server_stats.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u64),
                                  ctypes.POINTER(u64)]
    L.ss_server_destroy.argtypes = [vp]
    for name in ("ss_server_default_config", "ss_server_create", "ss_server_submit", "ss_server_poll",
                 "ss_server_drain", "ss_server_stats", "ss_server_destroy"):
        getattr(L, name).restype = ctypes.c_int


class Server:
    """ss_server: group-by requests served by concurrent lanes with packing of
    small semisort_= requests.  Inputs must be ready on the device when a
    request is submitted (the lanes do not wait for other streams); tensors
    handed to submit() are kept alive here until the request is polled done."""

    def __init__(self, device=0, lanes=None, pack_max_records=None, batch_records=None, hbm_budget=None,
                 params=None):
        L = lib()
        if not hasattr(L, "_server_bound"):
            _bind_server(L)
            L._server_bound = True
        cfg = ss_server_config()
        L.ss_server_default_config(ctypes.byref(cfg))
        for k, v in (("lanes", lanes), ("pack_max_records", pack_max_records), ("batch_records", batch_records),
                     ("hbm_budget", hbm_budget)):
            if v is not None:
                setattr(cfg, k, int(v))
        if params is not None:
            cfg.params = params
        self.h = ctypes.c_void_p()
        st = L.ss_server_create(int(device), ctypes.byref(cfg), ctypes.byref(self.h))
        if st != SS_OK:
            raise SemisortError(st, "ss_server_create failed")
        self._keep = {}

    def now(self):
        return lib().ss_server_now(self.h)

    def submit(self, op, keys, vals, out_a, out_b, arrival=0.0):
        req = ss_request()
        req.op = int(op)
        req.val_bytes = vals.element_size() if vals is not None else 8
        req.n = keys.numel()
        req.keys = keys.data_ptr()
        req.vals = vals.data_ptr() if vals is not None else None
        req.out_a = out_a.data_ptr()
        req.out_b = out_b.data_ptr()
        t = ctypes.c_uint64()
        st = lib().ss_server_submit(self.h, ctypes.byref(req), float(arrival), ctypes.byref(t))
        if st != SS_OK:
            raise SemisortError(st, "ss_server_submit rejected the request")
        self._keep[t.value] = (keys, vals, out_a, out_b)
        return t.value

    def poll(self, ticket):
        """(done, status, latency_s, m)."""
        done, res = ctypes.c_int(), ctypes.c_int()
        lat, m = ctypes.c_double(), ctypes.c_uint64()
        st = lib().ss_server_poll(self.h, ticket, ctypes.byref(done), ctypes.byref(res), ctypes.byref(lat),
                                  ctypes.byref(m))
        if st != SS_OK:
            raise SemisortError(st, "unknown ticket")
        if done.value:
            self._keep.pop(ticket, None)
        return bool(done.value), res.value, lat.value, m.value

    def drain(self):
        lib().ss_server_drain(self.h)

    def stats(self):
        c, calls, p, peak = (ctypes.c_uint64() for _ in range(4))
        lib().ss_server_stats(self.h, ctypes.byref(c), ctypes.byref(calls), ctypes.byref(p), ctypes.byref(peak))
        return {"completed": c.value, "calls": calls.value, "packed": p.value, "peak_reserved": peak.value}

    def close(self):
        if self.h:
            lib().ss_server_destroy(self.h)
            self.h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
