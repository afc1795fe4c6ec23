"""GPU parity for semisort_= : the HIP path (through the C-ABI) against the CPU
oracle, element by element after canonicalizing the free group order."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2304_10078_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2304_10078_amd import semisort as S  # noqa: E402
from tests.gpu_util import assert_semisort_equal, to_dev, to_host  # noqa: E402


def run_equal(keys, vals, params=None):
    ko, vo = S.semisort_equal(to_dev(keys), to_dev(vals), params=params)
    S.sync()  # waits and raises on a device-side error
    return to_host(ko, np.uint64), to_host(vo, vals.dtype)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_config1_uniform_1e5_keys_n_1e6():
    k, v = I.np_workload("uniform1e5_index", 10 ** 6, 1)
    _say("case: uniform1e5_index n=1e6 seed=1")
    ko, vo = run_equal(k, v)
    assert_semisort_equal(k, v, ko, vo, ctx="C1")


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 1000, 4095, 4096, 4097, 8191, 8193, 65537, 300001])
def test_ragged_sizes_small_key_range(n):
    rng = np.random.default_rng(n)
    k = rng.integers(0, max(2, n // 7), n, dtype=np.int64).astype(np.uint64)
    v = np.arange(n, dtype=np.uint64)
    _say(f"case: ragged n={n}")
    ko, vo = run_equal(k, v)
    assert_semisort_equal(k, v, ko, vo, ctx=f"n={n}")


@pytest.mark.parametrize("name,n", [("zipf1.2_hashed", 2_000_003), ("uniform1e9", 3_000_001),
                                    ("uniform1e3", 1_000_000), ("exp1e-5_u32idx", 1_500_000),
                                    ("zipf0.8_1e8_u32idx", 1_200_000)])
def test_paper_distributions(name, n):
    k, v = I.np_workload(name, n, 11)
    _say(f"case: {name} n={n}")
    ko, vo = run_equal(k, v)
    assert_semisort_equal(k, v, ko, vo, ctx=name)


def test_all_equal_and_all_distinct():
    n = 200_000
    k = np.full(n, 0xDEADBEEF, dtype=np.uint64)
    v = np.arange(n, dtype=np.uint64)
    _say("case: all equal")
    ko, vo = run_equal(k, v)
    assert np.array_equal(ko, k) and np.array_equal(vo, v)
    k = np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    _say("case: all distinct")
    ko, vo = run_equal(k, v)
    assert_semisort_equal(k, v, ko, vo, ctx="distinct")


def test_identity_hash_mode():
    k, v = I.np_workload("zipf0.8_1e8_u32idx", 500_000, 3)
    p = S.default_params(hash_mode="identity")
    _say("case: identity hash")
    ko, vo = run_equal(k, v, p)
    assert_semisort_equal(k, v, ko, vo, mode=O.HASH_IDENTITY, ctx="identity")


def test_small_parameters_force_deep_recursion():
    # n_L = 2 and alpha = 64 force many levels and many base cases
    rng = np.random.default_rng(5)
    n = 150_000
    k = rng.integers(0, 40_000, n, dtype=np.int64).astype(np.uint64)
    v = rng.integers(0, 2 ** 63, n, dtype=np.int64).astype(np.uint64)
    p = S.default_params(n_light_log2=1, base_case=64, sample_mult=20)
    _say("case: deep recursion")
    ko, vo = run_equal(k, v, p)
    assert_semisort_equal(k, v, ko, vo, ctx="deep")


def test_in_place_and_u32_values():
    k, v = I.np_workload("exp1e-5_u32idx", 700_000, 8)
    kd, vd = to_dev(k), to_dev(v)
    _say("case: in place u32")
    S.semisort_equal(kd, vd, keys_out=kd, vals_out=vd)
    S.sync()  # waits and raises on a device-side error
    assert_semisort_equal(k, v, to_host(kd, np.uint64), to_host(vd, np.uint32), ctx="inplace")


def test_deterministic_for_a_seed():
    k, v = I.np_workload("zipf1.2_hashed", 1_000_000, 2)
    a = run_equal(k, v)
    b = run_equal(k, v)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_empty_input_is_a_no_op():
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    ko, vo = S.semisort_equal(e, e)
    assert ko.numel() == 0


def test_rejects_overlapping_output():
    k = torch.zeros(100, dtype=torch.int64, device="cuda")
    v = torch.zeros(100, dtype=torch.int64, device="cuda")
    with pytest.raises(S.SemisortError):
        S.semisort_equal(k, v, keys_out=v, vals_out=k)


@pytest.mark.parametrize("name,n,c,tau", [("zipf1.2_hashed", 400_000, 300, 0), ("zipf1.2_hashed", 400_000, 1500, 2),
                                          ("uniform1e3", 400_000, 1200, 0), ("uniform1e3", 400_000, 1200, 3),
                                          ("zipf1.2_hashed", 20_000, 800, 3), ("zipf1.2_hashed", 5_000, 800, 3),
                                          ("zipf1.2_hashed", 50_000, 800, 3), ("uniform1e3", 9_000, 800, 2)])
def test_partition_matches_the_oracle_stage_model(name, n, c, tau):
    # One level of Steps 1-2 against the oracle's step-by-step model with the
    # same seed: heavy set and ids, bucket offsets and the distributed array T.
    # The uniform[0, 10^3) cases and the low thresholds put more than 512 keys
    # over the threshold, so the bounded-table rule decides the heavy set; the
    # sizes cover every sample size class (|S| padded to 1K, 2K, 4K, 8K, 16K).
    k, v = I.np_workload(name, n, 9)
    p = S.default_params(n_light_log2=6, sample_mult=c, heavy_min=tau)
    _say(f"case: partition n={n} {name} c={c} tau={tau}")
    tk, tv, off, hv = S.partition_equal(to_dev(k), to_dev(v), params=p)
    S.sync()  # waits and raises on a device-side error
    s = O.sample_size(n, p.sample_mult)
    idx = np.array([O.lib().orc_sample_index(p.seed, 0, 0, n, i) for i in range(s)], dtype=np.uint64)
    heavy = O.select_heavy(k[idx], tau or O.heavy_threshold(n), max_heavy=512)
    want_h = np.array([O.hash64(int(x)) for x in heavy], dtype=np.uint64)
    assert np.array_equal(to_host(hv, np.uint64), want_h)
    bids = O.bucket_ids(k, heavy, p.n_light_log2, 0)
    nb = (1 << p.n_light_log2) + heavy.size
    C = O.count_matrix(bids, 65536, nb)
    X, offs = O.column_prefix(C, n)
    ok, ov = O.distribute(k, v, bids, 65536, nb, X)
    assert np.array_equal(to_host(off, np.uint64), offs)
    assert np.array_equal(to_host(tk, np.uint64), ok)
    assert np.array_equal(to_host(tv, np.uint64), ov)


def test_batch_matches_each_instance_alone():
    rng = np.random.default_rng(21)
    sizes = [0, 1, 2, 100, 4095, 4096, 10_000, 70_000, 3, 250_000]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    n = int(offs[-1])
    k = np.empty(n, dtype=np.uint64)
    for i, sz in enumerate(sizes):
        a, b = int(offs[i]), int(offs[i + 1])
        k[a:b] = rng.integers(0, max(1, sz // 5), sz, dtype=np.int64).astype(np.uint64)
    v = np.arange(n, dtype=np.uint64)
    _say("case: batch of 10")
    ko, vo = S.semisort_equal_batch(to_dev(k), to_dev(v), offs)
    S.sync()  # waits and raises on a device-side error
    ko, vo = to_host(ko, np.uint64), to_host(vo, np.uint64)
    for i in range(len(sizes)):
        a, b = int(offs[i]), int(offs[i + 1])
        assert_semisort_equal(k[a:b], v[a:b], ko[a:b], vo[a:b], ctx=f"instance {i}")
        if b > a:
            ak, av = run_equal(k[a:b], v[a:b])
            assert np.array_equal(ak, ko[a:b]) and np.array_equal(av, vo[a:b]), f"instance {i} differs from alone"


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5])
def test_every_distribution_variant_gives_the_same_result(variant):
    ctx = S.context(0)
    try:
        for name, n in [("zipf1.2_hashed", 1_500_001), ("uniform1e9", 2_000_003),
                        ("exp1e-5_u32idx", 1_000_003), ("uniform1e3", 700_001)]:
            k, v = I.np_workload(name, n, 13)
            ctx.set_option(ctx.OPT_DIST_VARIANT, 0)
            ref = run_equal(k, v)
            ctx.set_option(ctx.OPT_DIST_VARIANT, variant)
            _say(f"case: variant {variant} {name} n={n}")
            ko, vo = run_equal(k, v)
            assert_semisort_equal(k, v, ko, vo, ctx=f"variant {variant} {name}")
            assert np.array_equal(ko, ref[0]) and np.array_equal(vo, ref[1])
    finally:
        ctx.set_option(ctx.OPT_DIST_VARIANT, 0)


def test_batched_configuration_shape_matches_the_oracle():
    # The batched configuration in miniature: log-uniform sizes (clamped at
    # 10^3), each instance with its own distribution among uniform[0, n/10),
    # Zipf 0.8 and 1.2 (hashed) and uniform[0, 100).
    k, v, offs, d = I.np_batch_workload(192, 1e3, 1e5, 3e6, 7)
    _say(f"case: batch of 192, n={k.size}")
    ko, vo = S.semisort_equal_batch(to_dev(k), to_dev(v), offs)
    S.sync()
    ko, vo = to_host(ko, np.uint64), to_host(vo, np.uint64)
    for i in range(192):
        a, b = int(offs[i]), int(offs[i + 1])
        assert_semisort_equal(k[a:b], v[a:b], ko[a:b], vo[a:b], ctx=f"instance {i} dist {d[i]}")


def test_autotuner_returns_a_grid_point_and_a_correct_result():
    k, v, offs, d = I.np_batch_workload(48, 1e3, 3e4, 5e5, 11)
    _say(f"case: autotune on a batch of 48, n={k.size}")
    best, ms = S.autotune_equal_batch(to_dev(k), to_dev(v), offs, reps=1)
    assert ms > 0
    assert best.sample_mult in (500, 800) and best.heavy_min in (0, 3) and best.n_light_log2 in (8, 10)
    assert best.base_case in (2048, 4096) and best.tile_max in (32768, 65536)
    ko, vo = S.semisort_equal_batch(to_dev(k), to_dev(v), offs, params=best)
    S.sync()
    ko, vo = to_host(ko, np.uint64), to_host(vo, np.uint64)
    for i in range(48):
        a, b = int(offs[i]), int(offs[i + 1])
        assert_semisort_equal(k[a:b], v[a:b], ko[a:b], vo[a:b], ctx=f"tuned instance {i}")


def test_tuned_batches_reuse_the_parameters_of_their_class():
    ctx = S.Context(0)
    try:
        assert S.autotune_cache(ctx=ctx) == 0
        k, v, offs, d = I.np_batch_workload(48, 1e3, 3e4, 5e5, 12)
        kd, vd = to_dev(k), to_dev(v)
        _say(f"case: tuned batch (first of its class), n={k.size}")
        ko, vo, used, now = S.semisort_equal_batch_tuned(kd, vd, offs, ctx=ctx)
        ctx.sync()
        assert now and S.autotune_cache(ctx=ctx) == 1
        first = (used.sample_mult, used.heavy_min, used.n_light_log2, used.base_case, used.tile_max)
        hk, hv = to_host(ko, np.uint64), to_host(vo, np.uint64)
        for i in range(48):
            a, b = int(offs[i]), int(offs[i + 1])
            assert_semisort_equal(k[a:b], v[a:b], hk[a:b], hv[a:b], ctx=f"tuned instance {i}")
        # another batch of the same class: no tuning, the same parameters,
        # the result of the plain batch call with them
        # (the same instance sizes, other keys)
        k2, v2, offs2 = k[::-1].copy(), v, offs
        _say("case: tuned batch (same class)")
        ko2, vo2, used2, now2 = S.semisort_equal_batch_tuned(to_dev(k2), to_dev(v2), offs2, ctx=ctx)
        rk, rv = S.semisort_equal_batch(to_dev(k2), to_dev(v2), offs2, params=used2, ctx=ctx)
        ctx.sync()
        assert not now2 and S.autotune_cache(ctx=ctx) == 1
        assert (used2.sample_mult, used2.heavy_min, used2.n_light_log2, used2.base_case, used2.tile_max) == first
        assert torch.equal(ko2, rk) and torch.equal(vo2, rv)
        # a batch of another size class is tuned on its own
        k3, v3, offs3, _ = I.np_batch_workload(8, 1e3, 3e3, 2e4, 14)
        _say("case: tuned batch (another class)")
        S.semisort_equal_batch_tuned(to_dev(k3), to_dev(v3), offs3, ctx=ctx)
        ctx.sync()
        assert S.autotune_cache(ctx=ctx) == 2
        assert S.autotune_cache(clear=True, ctx=ctx) == 0
    finally:
        ctx.close()


@pytest.mark.parametrize("t0,td", [(8192, 8192), (65536, 65536), (16384, 65536)])
def test_subarray_limits_do_not_change_the_result(t0, td):
    """The output of semisort_= depends only on the buckets and the input
    order, not on how levels are cut into subarrays: every setting of the
    per-level subarray limits gives the default's bytes."""
    ctx = S.context(0)
    try:
        for name, n in [("zipf1.2_hashed", 1_200_001), ("uniform1e9", 1_500_007)]:
            k, v = I.np_workload(name, n, 21)
            ref = run_equal(k, v)
            ctx.set_option(ctx.OPT_TILE0, t0)
            ctx.set_option(ctx.OPT_TILE_DEEP, td)
            _say(f"case: tiles {t0}/{td} {name} n={n}")
            ko, vo = run_equal(k, v)
            assert np.array_equal(ko, ref[0]) and np.array_equal(vo, ref[1]), f"{name} tiles {t0}/{td}"
    finally:
        ctx.set_option(ctx.OPT_TILE0, 0)
        ctx.set_option(ctx.OPT_TILE_DEEP, 0)
