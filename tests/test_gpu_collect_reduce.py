"""GPU parity for collect-reduce and histogram (Section 3.5): the HIP path
(through the C-ABI) against the CPU oracle.  The unordered calls return the
m pairs in an unspecified order, so both sides are compared after sorting by
key; keys are unique on both sides, so the sorted pairs must match exactly.
The ordered calls must match the oracle's ascending pairs as they stand."""
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
from tests.gpu_util import to_dev, to_host  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sorted_pairs(k, v):
    o = np.argsort(k, kind="stable")
    return k[o], v[o]


def check_cr(keys, vals, params=None, ctx=""):
    gk, gs = S.collect_reduce(to_dev(keys), to_dev(vals), params=params)
    S.sync()  # waits and raises on a device-side error
    gk, gs = _sorted_pairs(to_host(gk, np.uint64), to_host(gs, np.uint64))
    rk, rs = O.collect_reduce(keys, vals)
    assert gk.size == rk.size, f"{ctx}: {gk.size} groups, oracle {rk.size}"
    assert np.array_equal(gk, rk), f"{ctx}: keys differ"
    if not np.array_equal(gs, rs):
        i = int(np.nonzero(gs != rs)[0][0])
        raise AssertionError(f"{ctx}: sum of key {rk[i]} is {gs[i]}, oracle {rs[i]}")


def check_hist(keys, params=None, ctx=""):
    gk, gc = S.histogram(to_dev(keys), params=params)
    S.sync()  # waits and raises on a device-side error
    gk, gc = _sorted_pairs(to_host(gk, np.uint64), to_host(gc, np.uint64))
    rk, rc = O.histogram(keys)
    assert gk.size == rk.size, f"{ctx}: {gk.size} groups, oracle {rk.size}"
    assert np.array_equal(gk, rk), f"{ctx}: keys differ"
    if not np.array_equal(gc, rc):
        i = int(np.nonzero(gc != rc)[0][0])
        raise AssertionError(f"{ctx}: count of key {rk[i]} is {gc[i]}, oracle {rc[i]}")


def test_config1_uniform_1e5_keys_n_1e6():
    k, v = I.np_workload("uniform1e5_index", 10 ** 6, 1)
    _say("case: CR uniform1e5_index n=1e6")
    check_cr(k, v, ctx="CR C1")
    _say("case: histogram uniform1e5_index n=1e6")
    check_hist(k, ctx="hist C1")


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 1000, 4095, 4096, 4097, 8193, 65537, 65536 * 3 + 7, 300001])
def test_ragged_sizes(n):
    rng = np.random.default_rng(n + 100)
    k = rng.integers(0, max(2, n // 7), n, dtype=np.int64).astype(np.uint64)
    v = rng.integers(0, 2 ** 63, n, dtype=np.int64).astype(np.uint64)
    _say(f"case: ragged CR/hist n={n}")
    check_cr(k, v, ctx=f"CR n={n}")
    check_hist(k, ctx=f"hist n={n}")


@pytest.mark.parametrize("name,n", [("zipf1.2_hashed", 2_000_003), ("uniform1e9", 3_000_001),
                                    ("uniform1e3", 1_000_000), ("exp1e-5_u32idx", 1_500_000),
                                    ("zipf0.8_1e8_u32idx", 1_200_000)])
def test_paper_distributions(name, n):
    k, v = I.np_workload(name, n, 17)
    v = v.astype(np.uint64)
    _say(f"case: CR/hist {name} n={n}")
    check_cr(k, v, ctx=f"CR {name}")
    check_hist(k, ctx=f"hist {name}")


def test_sums_wrap_modulo_2_64():
    n = 300_000
    rng = np.random.default_rng(3)
    k = rng.integers(0, 50, n, dtype=np.int64).astype(np.uint64)
    v = np.full(n, 0xFFFF_FFFF_FFFF_FFF0, dtype=np.uint64)
    _say("case: wrapping sums")
    check_cr(k, v, ctx="wrap")


def test_identity_hash_and_deep_recursion():
    k, v = I.np_workload("zipf0.8_1e8_u32idx", 500_000, 3)
    v = v.astype(np.uint64)
    _say("case: identity hash")
    check_cr(k, v, S.default_params(hash_mode="identity"), ctx="identity")
    rng = np.random.default_rng(5)
    n = 150_000
    k = rng.integers(0, 40_000, n, dtype=np.int64).astype(np.uint64)
    v = rng.integers(0, 2 ** 63, n, dtype=np.int64).astype(np.uint64)
    p = S.default_params(n_light_log2=1, base_case=64, sample_mult=20)
    _say("case: deep recursion")
    check_cr(k, v, p, ctx="deep")
    check_hist(k, p, ctx="deep hist")


def test_all_equal_and_all_distinct():
    n = 200_000
    k = np.full(n, 0xDEADBEEF, dtype=np.uint64)
    v = np.arange(n, dtype=np.uint64)
    _say("case: CR all equal")
    check_cr(k, v, ctx="all equal")
    check_hist(k, ctx="all equal hist")
    k = np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    _say("case: CR all distinct")
    check_cr(k, v, ctx="distinct")
    check_hist(k, ctx="distinct hist")


def test_deterministic_for_a_seed():
    k, v = I.np_workload("zipf1.2_hashed", 1_000_000, 2)
    a = S.collect_reduce(to_dev(k), to_dev(v))
    a = (to_host(a[0], np.uint64), to_host(a[1], np.uint64))
    b = S.collect_reduce(to_dev(k), to_dev(v))
    b = (to_host(b[0], np.uint64), to_host(b[1], np.uint64))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_empty_input():
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    gk, gs = S.collect_reduce(e, e)
    assert gk.numel() == 0 and gs.numel() == 0
    gk, gc = S.histogram(e)
    assert gk.numel() == 0


def test_rejects_overlapping_outputs():
    k = torch.zeros(100, dtype=torch.int64, device="cuda")
    v = torch.zeros(100, dtype=torch.int64, device="cuda")
    with pytest.raises(S.SemisortError):
        S.collect_reduce(k, v, out_keys=v)


def test_histogram_after_semisort_on_one_context_reuses_workspace():
    # the same context serves semisort and collect-reduce in turn
    k, v = I.np_workload("exp1e-5_u32idx", 800_000, 4)
    v = v.astype(np.uint64)
    ctx = S.context(0)
    _say("case: mixed calls on one context")
    for _ in range(2):
        ko, vo = S.semisort_equal(to_dev(k), to_dev(v), ctx=ctx)
        check_hist(k, ctx="mixed hist")
        check_cr(k, v, ctx="mixed CR")


def check_ordered(keys, vals=None, params=None, ctx=""):
    """The ordered forms against the oracle, element by element (the oracle
    emits keys ascending as uint64; the pairs are unique)."""
    if vals is None:
        gk, gv = S.histogram(to_dev(keys), params=params, ordered=True)
        rk, rv = O.histogram(keys)
    else:
        gk, gv = S.collect_reduce(to_dev(keys), to_dev(vals), params=params, ordered=True)
        rk, rv = O.collect_reduce(keys, vals)
    S.sync()
    gk, gv = to_host(gk, np.uint64), to_host(gv, np.uint64)
    assert gk.size == rk.size, f"{ctx}: {gk.size} groups, oracle {rk.size}"
    if not np.array_equal(gk, rk):
        i = int(np.nonzero(gk != rk)[0][0])
        raise AssertionError(f"{ctx}: key {i} is {gk[i]}, oracle {rk[i]}")
    assert np.array_equal(gv, rv), f"{ctx}: results differ"


@pytest.mark.parametrize("name,n", [("exp1e-5_u32idx", 1_500_000), ("zipf0.8_1e8_u32idx", 1_200_000),
                                    ("zipf1.2_hashed", 700_001), ("uniform1e9", 900_000)])
def test_ordered_results_paper_distributions(name, n):
    k, v = I.np_workload(name, n, 23)
    v = v.astype(np.uint64)
    _say(f"case: ordered hist/CR {name} n={n}")
    check_ordered(k, ctx=f"ordered hist {name}")
    check_ordered(k, v, ctx=f"ordered CR {name}")


@pytest.mark.parametrize("n", [1, 2, 3, 64, 4097, 65537, 300001])
def test_ordered_results_ragged_and_unsigned_order(n):
    rng = np.random.default_rng(n + 7)
    # keys over the whole uint64 range: the order must be unsigned
    k = rng.integers(0, max(2, n // 3), n, dtype=np.int64).astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    v = rng.integers(0, 2 ** 63, n, dtype=np.int64).astype(np.uint64)
    _say(f"case: ordered hist/CR ragged n={n}")
    check_ordered(k, ctx=f"ordered hist n={n}")
    check_ordered(k, v, ctx=f"ordered CR n={n}")
    same = np.full(n, 5, dtype=np.uint64)
    check_ordered(same, v, ctx=f"ordered CR one key n={n}")


def test_ordered_results_empty_and_small_parameters():
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    gk, gc = S.histogram(e, ordered=True)
    assert gk.numel() == 0 and gc.numel() == 0
    rng = np.random.default_rng(11)
    k = rng.integers(0, 30_000, 120_000, dtype=np.int64).astype(np.uint64)
    p = S.default_params(n_light_log2=2, base_case=256, sample_mult=20, tile_min=8192, tile_max=8192)
    _say("case: ordered histogram, small parameters")
    check_ordered(k, params=p, ctx="ordered hist small params")


def check_monoid(keys, vals, op, ordered=False, params=None, ctx=""):
    """collect-reduce with the min / max / xor / first / last / affine monoids
    against the oracle (first / last: the value of the key's first / last
    record in input order; affine: the composition of the key's maps in input
    order)."""
    gk, gv = S.collect_reduce(to_dev(keys), to_dev(vals), params=params, ordered=ordered, op=op)
    S.sync()
    gk, gv = to_host(gk, np.uint64), to_host(gv, np.uint64)
    if not ordered:
        gk, gv = _sorted_pairs(gk, gv)
    rk, rv = O.collect_reduce(keys, vals, op=op)
    assert gk.size == rk.size, f"{ctx}: {gk.size} groups, oracle {rk.size}"
    assert np.array_equal(gk, rk), f"{ctx}: keys differ"
    if not np.array_equal(gv, rv):
        i = int(np.nonzero(gv != rv)[0][0])
        raise AssertionError(f"{ctx}: {op} of key {rk[i]} is {gv[i]}, oracle {rv[i]}")


def _wide_values(n, seed):
    # uint64 values over the whole range (the top bit decides unsigned min / max)
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2 ** 63, n, dtype=np.int64).astype(np.uint64) * np.uint64(2) + np.uint64(seed & 1)


def _affine_values(n, seed):
    # maps t -> a t + b mod 2^32 with ODD a: invertible, so every record of a
    # group changes its fold (with even multipliers the product of a few
    # dozen of them is 0 mod 2^32 and a long group's fold would depend only
    # on its last records, hiding a lost carry)
    return _wide_values(n, seed) | np.uint64(1 << 32)


def _monoid_values(op, n, seed):
    return _affine_values(n, seed) if op == "affine" else _wide_values(n, seed)


@pytest.mark.parametrize("op", ["min", "max", "xor", "first", "last", "affine"])
@pytest.mark.parametrize("name,n", [("zipf1.2_hashed", 1_500_001), ("uniform1e9", 1_000_000),
                                    ("uniform1e3", 700_000), ("exp1e-5_u32idx", 900_000)])
def test_monoids_paper_distributions(op, name, n):
    k, _ = I.np_workload(name, n, 31)
    v = _monoid_values(op, n, 5)
    _say(f"case: CR {op} {name} n={n}")
    check_monoid(k, v, op, ctx=f"CR {op} {name}")


@pytest.mark.parametrize("op", ["min", "max", "xor", "first", "last", "affine"])
def test_monoids_ragged_ordered_and_deep(op):
    for n in [1, 2, 3, 64, 4097, 65537, 200_003]:
        rng = np.random.default_rng(n)
        k = rng.integers(0, max(2, n // 6), n, dtype=np.int64).astype(np.uint64)
        v = _monoid_values(op, n, n)
        _say(f"case: CR {op} ragged n={n}")
        check_monoid(k, v, op, ctx=f"CR {op} n={n}")
        check_monoid(k, v, op, ordered=True, ctx=f"CR {op} ordered n={n}")
    rng = np.random.default_rng(9)
    n = 150_000
    k = rng.integers(0, 40_000, n, dtype=np.int64).astype(np.uint64)
    v = _monoid_values(op, n, 3)
    p = S.default_params(n_light_log2=1, base_case=64, sample_mult=20)
    _say(f"case: CR {op} deep recursion")
    check_monoid(k, v, op, params=p, ctx=f"CR {op} deep")
    k = np.full(n, 77, dtype=np.uint64)  # one key: a single heavy bucket
    check_monoid(k, v, op, ctx=f"CR {op} one key")


def test_affine_fold_carries_across_chunks_blocks_and_rounds():
    # The in-order fold carries the open fold across 4096-record chunks, then
    # across blocks of 256 chunks (2^20 positions), then across rounds of
    # block totals.  Groups long enough to straddle those boundaries, with
    # invertible maps, make every carry visible; rounds of 1 and 2 block
    # totals reach the cross-round carry at this size.
    n = 3 * (1 << 20) + 4099
    v = _affine_values(n, 17)
    cases = [("one key", np.full(n, 5, dtype=np.uint64)),
             ("seven keys", np.random.default_rng(3).integers(0, 7, n, dtype=np.int64).astype(np.uint64)),
             ("two keys in runs", (np.arange(n, dtype=np.uint64) // np.uint64(700_001)) % np.uint64(2)),
             ("zipf", I.np_workload("zipf1.2_hashed", n, 9)[0])]
    ctx = S.context(0)
    try:
        for rb in (1024, 2, 1):
            ctx.set_option(S.Context.OPT_FOLD_ROUND, rb)
            for name, k in cases:
                _say(f"case: CR affine {name} n={n} fold round {rb}")
                check_monoid(k, v, "affine", ctx=f"affine {name} round {rb}")
    finally:
        ctx.set_option(S.Context.OPT_FOLD_ROUND, 1024)


def test_affine_fold_rejects_a_bad_round():
    ctx = S.context(0)
    for bad in (0, 3, 2048):
        with pytest.raises(S.SemisortError):
            ctx.set_option(S.Context.OPT_FOLD_ROUND, bad)


def test_monoid_rejects_an_unknown_op():
    import ctypes
    k = torch.zeros(100, dtype=torch.int64, device="cuda")
    v = torch.zeros(100, dtype=torch.int64, device="cuda")
    ok, ov = torch.empty_like(k), torch.empty_like(k)
    m = ctypes.c_uint64()
    ctx = S.context(0)
    st = S.lib().ss_collect_reduce_monoid(ctx.h, S._ptr(k), S._ptr(v), 100, 7, 0, S._ptr(ok), S._ptr(ov),
                                          ctypes.byref(m), None)
    assert st == S.SS_EINVAL
