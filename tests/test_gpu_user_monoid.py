"""GPU parity of collect-reduce with a caller's monoid (ss_monoid_compile +
ss_collect_reduce_user): the source is compiled at run time into the in-order
segmented fold, run after a stable semisort_= (Section 3.5 defines
collect-reduce for any monoid; stability lets a non-commutative one fold in
input order).  Against the oracle: wrapping sums (u64 and u32 values), affine
maps with odd multipliers, products of 2 x 2 matrices mod 2^16 (not
commutative: every record and every carry changes the result), and a
(min, max) pair of 32-bit halves built by the map; groups that straddle
4096-record chunks, blocks of 256 chunks and rounds of block totals; ordered
output; empty and one-record inputs; sources that do not compile."""
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

SUM = """
typedef ss_u64 ss_t;
__device__ ss_t ss_identity() { return 0; }
__device__ ss_t ss_map(ss_u64 v) { return v; }
__device__ ss_t ss_combine(ss_t a, ss_t b) { return a + b; }
"""

AFFINE = """
// t -> a t + b mod 2^32 with (a, b) the high and low halves; a then b
struct ss_t { ss_u32 b, a; };
__device__ ss_t ss_identity() { return ss_t{0u, 1u}; }
__device__ ss_t ss_map(ss_u64 v) { return ss_t{(ss_u32)v, (ss_u32)(v >> 32)}; }
__device__ ss_t ss_combine(ss_t x, ss_t y) { return ss_t{y.a * x.b + y.b, y.a * x.a}; }
"""

MAT2 = """
// 2 x 2 matrices over the integers mod 2^16, entries from the value's 16-bit fields
struct ss_t { unsigned short a, b, c, d; };
__device__ ss_t ss_identity() { return ss_t{1, 0, 0, 1}; }
__device__ ss_t ss_map(ss_u64 v)
{
    return ss_t{(unsigned short)v, (unsigned short)(v >> 16), (unsigned short)(v >> 32), (unsigned short)(v >> 48)};
}
__device__ ss_t ss_combine(ss_t x, ss_t y)
{
    return ss_t{(unsigned short)(x.a * y.a + x.b * y.c), (unsigned short)(x.a * y.b + x.b * y.d),
                (unsigned short)(x.c * y.a + x.d * y.c), (unsigned short)(x.c * y.b + x.d * y.d)};
}
"""

MINMAX = """
// (min, max) of the value's low 32 bits
struct ss_t { ss_u32 lo, hi; };
__device__ ss_t ss_identity() { return ss_t{0xFFFFFFFFu, 0u}; }
__device__ ss_t ss_map(ss_u64 v) { return ss_t{(ss_u32)v, (ss_u32)v}; }
__device__ ss_t ss_combine(ss_t x, ss_t y) { return ss_t{x.lo < y.lo ? x.lo : y.lo, x.hi > y.hi ? x.hi : y.hi}; }
"""

_cache = {}


def _monoid(src):
    if src not in _cache:
        _cache[src] = S.Monoid(src)
    return _cache[src]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(k, v, src, ordered=False):
    gk, gv = S.collect_reduce_user(to_dev(k), to_dev(v), _monoid(src), ordered=ordered)
    S.sync()
    return to_host(gk, np.uint64), to_host(gv, np.uint64)


def _sorted(gk, gv):
    o = np.argsort(gk, kind="stable")
    return gk[o], gv[o]


def _check(k, v, src, op, ctx="", ordered=False):
    gk, gv = _run(k, v, src, ordered)
    if ordered:
        assert np.all(gk[1:] > gk[:-1]), f"{ctx}: keys not ascending"
    gk, gv = _sorted(gk, gv)
    v64 = v.astype(np.uint64)
    if op == "minmax":
        lo = v64 & np.uint64(0xFFFFFFFF)
        rk, rmin = O.collect_reduce(k, lo, op="min")
        _, rmax = O.collect_reduce(k, lo, op="max")
        rv = rmin | (rmax << np.uint64(32))
    else:
        rk, rv = O.collect_reduce(k, v64, op=op)
    assert np.array_equal(gk, rk), f"{ctx}: keys differ from the oracle"
    if not np.array_equal(gv, rv):
        i = int(np.nonzero(gv != rv)[0][0])
        raise AssertionError(f"{ctx}: fold of key {int(gk[i])} is {int(gv[i]):#x}, oracle {int(rv[i]):#x}")


def _values(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "affine":  # odd multipliers: every map is invertible, so every record shows
        a = rng.integers(0, 1 << 31, n, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
        b = rng.integers(0, 1 << 32, n, dtype=np.uint64)
        return (a << np.uint64(32)) | b
    if kind == "mat2":  # unimodular matrices (det 1, invertible): every record changes the product
        x = rng.integers(0, 1 << 16, n, dtype=np.uint64)
        y = rng.integers(0, 1 << 16, n, dtype=np.uint64)
        # (1, x; 0, 1)(1, 0; y, 1) = (1 + x y, x; y, 1)
        a = (np.uint64(1) + x * y) & np.uint64(0xFFFF)
        return a | (x << np.uint64(16)) | (y << np.uint64(32)) | (np.uint64(1) << np.uint64(48))
    return rng.integers(0, 2 ** 63, n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n, dtype=np.uint64)


@pytest.mark.parametrize("src,op", [(SUM, "sum"), (AFFINE, "affine"), (MAT2, "mat2"), (MINMAX, "minmax")],
                         ids=["sum", "affine", "mat2", "minmax"])
def test_user_monoids_on_the_paper_distributions(src, op):
    for name, n in (("zipf1.2_hashed", 1_500_007), ("uniform1e9", 1_000_003), ("uniform1e3", 700_001)):
        k, _ = I.np_workload(name, n, 71)
        v = _values(op, n, 72)
        _say(f"case: user monoid {op} {name} n={n}")
        _check(k, v, src, op, ctx=f"{op} {name}")
    _say(f"case: user monoid {op} ordered")
    k, _ = I.np_workload("zipf1.2_hashed", 300_001, 73)
    _check(k, _values(op, 300_001, 74), src, op, ctx=f"{op} ordered", ordered=True)


def test_user_monoid_with_32bit_values():
    k, _ = I.np_workload("zipf1.2_hashed", 900_001, 75)
    v32 = np.random.default_rng(76).integers(0, 1 << 32, 900_001, dtype=np.uint64).astype(np.uint32)
    _say("case: user sum with u32 values")
    gk, gv = _sorted(*_run(k, v32, SUM))
    rk, rv = O.collect_reduce(k, v32.astype(np.uint64), op="sum")
    assert np.array_equal(gk, rk) and np.array_equal(gv, rv)
    _say("case: user min/max with u32 values")
    _check(k, v32, MINMAX, "minmax", ctx="minmax u32")


def test_user_fold_carries_across_chunks_blocks_and_rounds():
    n = 3 * (1 << 20) + 4099
    v = _values("mat2", n, 77)
    cases = [("one key", np.full(n, 5, dtype=np.uint64)),
             ("seven keys", np.random.default_rng(3).integers(0, 7, n, dtype=np.int64).astype(np.uint64)),
             ("two keys in runs", (np.arange(n, dtype=np.uint64) // np.uint64(700_001)) % np.uint64(2))]
    ctx = S.context(0)
    try:
        for rb in (1024, 2, 1):
            ctx.set_option(S.Context.OPT_FOLD_ROUND, rb)
            for name, k in cases:
                _say(f"case: user mat2 {name} n={n} fold round {rb}")
                _check(k, v, MAT2, "mat2", ctx=f"mat2 {name} round {rb}")
    finally:
        ctx.set_option(S.Context.OPT_FOLD_ROUND, 1024)


def test_user_monoid_edge_cases():
    m = _monoid(MAT2)
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    gk, gv = S.collect_reduce_user(e, e, m)
    assert gk.numel() == 0 and gv.numel() == 0
    for n in (1, 2, 4095, 4096, 4097):
        k = np.random.default_rng(n).integers(0, 3, n, dtype=np.uint64)
        _check(k, _values("mat2", n, n + 1), MAT2, "mat2", ctx=f"n={n}")


def test_user_monoid_sources_that_do_not_compile():
    with pytest.raises(S.SemisortError) as e:
        S.Monoid("typedef ss_u64 ss_t;\n__device__ ss_t ss_identity() { return 0 }\n")
    assert "monoid" in str(e.value)
    # an element wider than 8 bytes
    with pytest.raises(S.SemisortError):
        S.Monoid("struct ss_t { ss_u64 a, b; };\n__device__ ss_t ss_identity() { return ss_t{0, 0}; }\n"
                 "__device__ ss_t ss_map(ss_u64 v) { return ss_t{v, v}; }\n"
                 "__device__ ss_t ss_combine(ss_t x, ss_t y) { return x; }\n")
