"""Host-side checks of the C-ABI library: it loads without a GPU, exports every
entry point include/semisort.h declares, and its argument checks refuse bad
calls before touching a device."""
import ctypes
import os

import pytest

from paper_2304_10078_amd import semisort as S


def _lib_or_skip():
    if not os.path.exists(S.LIB_PATH):
        pytest.skip("libsemisort_hip.so not built")
    return S.lib()


def test_header_declares_the_boundary():
    names = S.declared_symbols()
    for want in ["ss_create", "ss_destroy", "ss_semisort_equal", "ss_semisort_equal_batch",
                 "ss_semisort_less", "ss_semisort_less_batch", "ss_collect_reduce", "ss_histogram",
                 "ss_collect_reduce_ordered", "ss_histogram_ordered", "ss_collect_reduce_monoid",
                 "ss_transpose_csr", "ss_semisort_equal_batch_capturable",
                 "ss_autotune_equal_batch", "ss_server_create", "ss_server_submit", "ss_server_poll",
                 "ss_server_drain", "ss_server_stats", "ss_server_destroy", "ss_server_now",
                 "ss_partition_equal", "ss_default_params", "ss_last_error", "ss_sync",
                 "ss_semisort_equal_batch_noalloc", "ss_batch", "ss_collect_reduce_async", "ss_histogram_async",
                 "ss_workspace_bytes", "ss_workspace_held", "ss_semisort_equal_keys", "ss_semisort_less_keys",
                 "ss_monoid_compile", "ss_monoid_destroy", "ss_collect_reduce_user",
                 "ss_semisort_equal_batch_tuned", "ss_autotune_cache"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    missing = [n for n in S.declared_symbols() if not hasattr(L, n)]
    assert not missing, missing


def test_default_params():
    _lib_or_skip()
    p = S.default_params()
    assert (p.n_light_log2, p.base_case, p.sample_mult, p.heavy_min) == (10, 4096, 800, 3)
    assert p.tile_min == 8192 and p.tile_max == 0 and p.hash_mode == S.HASH_MIX64


def test_null_context_is_rejected():
    L = _lib_or_skip()
    assert L.ss_semisort_equal(None, None, None, 8, 10, None, None, None) == S.SS_EINVAL
    assert L.ss_semisort_less(None, None, None, 8, 10, None, None, None) == S.SS_EINVAL
    m = ctypes.c_uint64(7)
    assert L.ss_collect_reduce(None, None, None, 10, None, None, ctypes.byref(m), None) == S.SS_EINVAL
    assert L.ss_histogram(None, None, 10, None, None, ctypes.byref(m), None) == S.SS_EINVAL
    assert L.ss_collect_reduce_ordered(None, None, None, 10, None, None, ctypes.byref(m), None) == S.SS_EINVAL
    assert L.ss_histogram_ordered(None, None, 10, None, None, ctypes.byref(m), None) == S.SS_EINVAL
    assert L.ss_collect_reduce_monoid(None, None, None, 10, 1, 0, None, None, ctypes.byref(m), None) == S.SS_EINVAL
    assert L.ss_transpose_csr(None, 4, 10, None, None, None, None, None) == S.SS_EINVAL
    assert L.ss_semisort_equal_batch_capturable(None, None, None, 8, None, 1, 10, None, None, 4, None) == S.SS_EINVAL
    assert L.ss_semisort_equal_batch_noalloc(None, None, None, 8, None, 1, 10, None, None, 4, None) == S.SS_EINVAL
    assert L.ss_collect_reduce_async(None, None, None, 10, 0, 0, None, None, None, None) == S.SS_EINVAL
    assert L.ss_histogram_async(None, None, 10, 0, None, None, None, None) == S.SS_EINVAL
    assert L.ss_batch(None, None, 1, None) == S.SS_EINVAL
    assert L.ss_workspace_held(None, None) == S.SS_EINVAL
    assert L.ss_semisort_equal_keys(None, None, 16, None, 8, 10, None, None, None) == S.SS_EINVAL
    assert L.ss_semisort_less_keys(None, None, 4, None, 8, 10, None, None, None) == S.SS_EINVAL
    h = ctypes.c_void_p()
    assert L.ss_monoid_compile(None, b"typedef ss_u64 ss_t;", ctypes.byref(h)) == S.SS_EINVAL and not h.value
    assert L.ss_monoid_destroy(None) == S.SS_EINVAL
    assert L.ss_semisort_equal_batch_tuned(None, None, None, 8, None, 1, None, None, None, None) == S.SS_EINVAL
    assert L.ss_autotune_cache(None, 1, None) == S.SS_EINVAL
    assert L.ss_collect_reduce_user(None, None, None, None, 8, 10, 0, None, None, ctypes.byref(m), None) == S.SS_EINVAL
    assert L.ss_destroy(None) == S.SS_EINVAL
    assert L.ss_sync(None) == S.SS_EINVAL
    assert L.ss_last_error(None) == b"null context"


def test_create_without_a_device_fails_cleanly():
    L = _lib_or_skip()
    h = ctypes.c_void_p()
    st = L.ss_create(999, None, 0, ctypes.byref(h))
    assert st == S.SS_EINVAL and not h.value


def test_server_without_a_device_fails_cleanly():
    L = _lib_or_skip()
    import paper_2304_10078_amd.semisort as SS
    with pytest.raises(SS.SemisortError):
        SS.Server(device=999)
    assert L.ss_server_destroy(None) == S.SS_EINVAL


def test_workspace_planning_query():
    # the planning bound needs no device: it grows with n, covers the n-sized
    # buffers the engine must hold (temporary keys and values, bucket ids),
    # and refuses what the calls refuse
    _lib_or_skip()
    for op, vb in ((S.OP_SEMISORT_EQUAL, 8), (S.OP_SEMISORT_EQUAL, 4), (S.OP_SEMISORT_LESS, 8),
                   (S.OP_HISTOGRAM, 8), (S.OP_COLLECT_REDUCE, 8)):
        prev = 0
        for n in (0, 1, 4095, 4096, 10 ** 5, 10 ** 7, 10 ** 9, (1 << 31) - 1):
            b = S.workspace_bound(op, n, vb)
            assert b >= prev, (op, n)
            assert b >= n * (8 + vb + 2), (op, n)
            prev = b
        assert S.workspace_bound(op, 0, vb) == 0
        assert S.workspace_bound(op, 10 ** 9, vb) < 100 * 10 ** 9
    # a smaller base case means more subproblems per level, so a larger bound
    small = S.default_params(base_case=256)
    assert S.workspace_bound(S.OP_SEMISORT_EQUAL, 10 ** 7, 8, small) > S.workspace_bound(S.OP_SEMISORT_EQUAL, 10 ** 7)
    for bad in ((7, 100, 8), (S.OP_SEMISORT_EQUAL, 100, 2), (S.OP_SEMISORT_LESS, 1 << 31, 8)):
        with pytest.raises(S.SemisortError):
            S.workspace_bound(*bad)
    with pytest.raises(S.SemisortError):
        S.workspace_bound(S.OP_SEMISORT_EQUAL, 100, 8, S.default_params(base_case=10))
