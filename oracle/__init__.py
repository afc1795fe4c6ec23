"""CPU oracle for semisort, histogram and collect-reduce -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (plain C,
single-threaded, see ``oracle.h``) with numpy marshalling.  Nothing here shares
code with the GPU library.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        u64, u32, i64, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int
        vp = ctypes.c_void_p
        L.orc_hash.restype = u64
        L.orc_hash.argtypes = [u64, i32]
        L.orc_splitmix_mix.restype = u64
        L.orc_splitmix_mix.argtypes = [u64]
        L.orc_semisort_equal.restype = i32
        L.orc_semisort_equal.argtypes = [vp, vp, u32, u64, i32, vp, vp]
        L.orc_semisort_less.restype = i32
        L.orc_semisort_less.argtypes = [vp, vp, u32, u64, vp, vp]
        L.orc_histogram.restype = i64
        L.orc_histogram.argtypes = [vp, u64, vp, vp]
        L.orc_collect_reduce.restype = i64
        L.orc_collect_reduce.argtypes = [vp, vp, u64, vp, vp]
        L.orc_transpose_csr.restype = ctypes.c_int
        L.orc_transpose_csr.argtypes = [u64, u64, vp, vp, vp, vp]
        L.orc_collect_reduce_monoid.restype = i64
        L.orc_collect_reduce_monoid.argtypes = [vp, vp, u64, ctypes.c_int, vp, vp]
        L.orc_semisort_equal_wide.restype = i32
        L.orc_semisort_equal_wide.argtypes = [vp, vp, u32, u64, vp, vp]
        L.orc_canonicalize_equal_wide.restype = i64
        L.orc_canonicalize_equal_wide.argtypes = [vp, vp, u32, u64, vp, vp]
        L.orc_canonicalize_equal.restype = i64
        L.orc_canonicalize_equal.argtypes = [vp, vp, u32, u64, i32, vp, vp]
        L.orc_stats.restype = i32
        L.orc_stats.argtypes = [vp, u64, ctypes.c_double, vp, vp, vp]
        L.orc_sample_size.restype = u32
        L.orc_sample_size.argtypes = [u64, u32]
        L.orc_heavy_threshold.restype = u32
        L.orc_heavy_threshold.argtypes = [u64]
        L.orc_sample_index.restype = u64
        L.orc_sample_index.argtypes = [u64, u32, u64, u64, u64]
        L.orc_select_heavy.restype = i64
        L.orc_select_heavy.argtypes = [vp, u32, u32, i32, u32, vp]
        L.orc_bucket_ids.restype = None
        L.orc_bucket_ids.argtypes = [vp, u64, vp, u32, u32, u32, i32, vp]
        L.orc_count_matrix.restype = None
        L.orc_count_matrix.argtypes = [vp, u64, u64, u32, vp]
        L.orc_column_prefix.restype = None
        L.orc_column_prefix.argtypes = [vp, u64, u32, u64, vp, vp]
        L.orc_distribute.restype = None
        L.orc_distribute.argtypes = [vp, vp, u32, vp, u64, u64, u32, vp, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else ctypes.c_void_p(0)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def _vals(v):
    v = np.ascontiguousarray(v)
    if v.dtype not in (np.uint64, np.uint32):
        raise TypeError("values must be uint64 or uint32")
    return v, v.dtype.itemsize


HASH_MIX64 = 0
HASH_IDENTITY = 1


def hash64(k, mode=HASH_MIX64):
    return int(lib().orc_hash(int(k), mode))


def splitmix_mix(z):
    return int(lib().orc_splitmix_mix(int(z)))


def semisort_equal(keys, vals, hash_mode=HASH_MIX64):
    keys = _u64(keys)
    vals, vb = _vals(vals)
    ko = np.empty_like(keys)
    vo = np.empty_like(vals)
    if lib().orc_semisort_equal(_p(keys), _p(vals), vb, keys.size, hash_mode, _p(ko), _p(vo)) != 0:
        raise MemoryError("oracle semisort_equal")
    return ko, vo


def semisort_less(keys, vals):
    keys = _u64(keys)
    vals, vb = _vals(vals)
    ko = np.empty_like(keys)
    vo = np.empty_like(vals)
    if lib().orc_semisort_less(_p(keys), _p(vals), vb, keys.size, _p(ko), _p(vo)) != 0:
        raise MemoryError("oracle semisort_less")
    return ko, vo


def histogram(keys):
    keys = _u64(keys)
    ok = np.empty_like(keys)
    oc = np.empty_like(keys)
    m = lib().orc_histogram(_p(keys), keys.size, _p(ok), _p(oc))
    if m < 0:
        raise MemoryError("oracle histogram")
    return ok[:m].copy(), oc[:m].copy()


MONOIDS = {"sum": 0, "min": 1, "max": 2, "xor": 3, "first": 4, "last": 5, "affine": 6, "mat2": 7}


def collect_reduce(keys, vals, op="sum"):
    """(unique keys ascending, fold of their values); op one of MONOIDS."""
    keys = _u64(keys)
    vals = _u64(vals)
    ok = np.empty_like(keys)
    os_ = np.empty_like(keys)
    if op == "sum":
        m = lib().orc_collect_reduce(_p(keys), _p(vals), keys.size, _p(ok), _p(os_))
    else:
        m = lib().orc_collect_reduce_monoid(_p(keys), _p(vals), keys.size, MONOIDS[op], _p(ok), _p(os_))
    if m < 0:
        raise MemoryError("oracle collect_reduce")
    return ok[:m].copy(), os_[:m].copy()


def transpose_csr(offs, cols):
    """Transposed CSR (offsets uint64[nv + 1], cols uint32[ne]) of the graph
    with offsets `offs` (nv + 1 entries) and targets `cols` (uint32)."""
    offs = np.ascontiguousarray(offs, dtype=np.uint64)
    cols = np.ascontiguousarray(cols, dtype=np.uint32)
    nv, ne = offs.size - 1, cols.size
    oo = np.empty(nv + 1, dtype=np.uint64)
    oc = np.empty(max(ne, 1), dtype=np.uint32)
    r = lib().orc_transpose_csr(nv, ne, _p(offs), _p(cols), _p(oo), _p(oc))
    if r == -2:
        raise ValueError("invalid CSR")
    if r != 0:
        raise MemoryError("oracle transpose_csr")
    return oo, oc[:ne].copy()


def canonicalize_equal(keys, vals, hash_mode=HASH_MIX64):
    """Returns (bad, canon_keys, canon_vals); bad == -1 when equal keys are contiguous."""
    keys = _u64(keys)
    vals, vb = _vals(vals)
    ck = np.empty_like(keys)
    cv = np.empty_like(vals)
    bad = lib().orc_canonicalize_equal(_p(keys), _p(vals), vb, keys.size, hash_mode, _p(ck), _p(cv))
    if bad == -2:
        raise MemoryError("oracle canonicalize")
    return int(bad), ck, cv


def _wide(keys):
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    if k.ndim != 2 or k.shape[1] != 2:
        raise ValueError("128-bit keys are an (n, 2) uint64 array of (low, high) words")
    return k


def semisort_equal_wide(keys, vals):
    """Stable semisort of 128-bit keys ((n, 2) uint64: low, high words), groups
    in ascending key order."""
    keys = _wide(keys)
    vals, vb = _vals(vals)
    ko = np.empty_like(keys)
    vo = np.empty_like(vals)
    if lib().orc_semisort_equal_wide(_p(keys), _p(vals), vb, keys.shape[0], _p(ko), _p(vo)) != 0:
        raise MemoryError("oracle semisort_equal_wide")
    return ko, vo


def canonicalize_equal_wide(keys, vals):
    """Returns (bad, canon_keys, canon_vals) for 128-bit keys; bad == -1 when
    equal keys are contiguous."""
    keys = _wide(keys)
    vals, vb = _vals(vals)
    ck = np.empty_like(keys)
    cv = np.empty_like(vals)
    bad = lib().orc_canonicalize_equal_wide(_p(keys), _p(vals), vb, keys.shape[0], _p(ck), _p(cv))
    if bad == -2:
        raise MemoryError("oracle canonicalize_equal_wide")
    return int(bad), ck, cv


def stats(keys, heavy_threshold):
    keys = _u64(keys)
    d = ctypes.c_uint64()
    mx = ctypes.c_uint64()
    hv = ctypes.c_uint64()
    if lib().orc_stats(_p(keys), keys.size, float(heavy_threshold), ctypes.byref(d), ctypes.byref(mx), ctypes.byref(hv)) != 0:
        raise MemoryError("oracle stats")
    return int(d.value), int(mx.value), int(hv.value)


def sample_size(n, c=500):
    return int(lib().orc_sample_size(int(n), int(c)))


def heavy_threshold(n):
    return int(lib().orc_heavy_threshold(int(n)))


def sample_indices(seed, level, start, length, count):
    L = lib()
    return np.array([L.orc_sample_index(seed, level, start, length, i) for i in range(count)], dtype=np.uint64)


def select_heavy(sample_keys, tau, hash_mode=HASH_MIX64, max_heavy=1 << 16):
    s = _u64(sample_keys)
    out = np.empty(max(1, min(max_heavy, s.size)), dtype=np.uint64)
    nh = lib().orc_select_heavy(_p(s), s.size, int(tau), hash_mode, out.size, _p(out))
    if nh < 0:
        raise MemoryError("oracle select_heavy")
    return out[:nh].copy()


def bucket_ids(keys, heavy_keys, nl_bits, shift, hash_mode=HASH_MIX64):
    keys = _u64(keys)
    hk = _u64(heavy_keys)
    b = np.empty(keys.size, dtype=np.uint32)
    lib().orc_bucket_ids(_p(keys), keys.size, _p(hk), hk.size, nl_bits, shift, hash_mode, _p(b))
    return b


def count_matrix(bids, tile, nb):
    bids = np.ascontiguousarray(bids, dtype=np.uint32)
    tiles = (bids.size + tile - 1) // tile
    C = np.zeros((tiles, nb), dtype=np.uint32)
    lib().orc_count_matrix(_p(bids), bids.size, tile, nb, _p(C))
    return C


def column_prefix(C, n):
    C = np.ascontiguousarray(C, dtype=np.uint32)
    tiles, nb = C.shape
    X = np.zeros_like(C)
    off = np.zeros(nb + 1, dtype=np.uint64)
    lib().orc_column_prefix(_p(C), tiles, nb, n, _p(X), _p(off))
    return X, off


def distribute(keys, vals, bids, tile, nb, X):
    keys = _u64(keys)
    vals, vb = _vals(vals)
    bids = np.ascontiguousarray(bids, dtype=np.uint32)
    X = np.ascontiguousarray(X, dtype=np.uint32)
    tk = np.zeros_like(keys)
    tv = np.zeros_like(vals)
    lib().orc_distribute(_p(keys), _p(vals), vb, _p(bids), keys.size, tile, nb, _p(X), _p(tk), _p(tv))
    return tk, tv
