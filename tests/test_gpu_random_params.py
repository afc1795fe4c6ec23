"""Randomized GPU parity: many small inputs, each with its own size, key
distribution, value width and parameter set (light-bucket bits, base-case
threshold, sample multiplier, heavy threshold, subarray limits, hash mode),
run through every operation and compared with the oracle.  The fixed tests
pin each feature; this one looks for interactions between them."""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2304_10078_amd import semisort as S  # noqa: E402
from tests.gpu_util import assert_semisort_equal, to_dev, to_host  # noqa: E402

CASES = 24


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _keys(rng, n):
    kind = int(rng.integers(0, 5))
    if kind == 0:  # few distinct keys: heavy buckets
        k = rng.integers(0, int(rng.integers(1, 50)), n, dtype=np.int64)
    elif kind == 1:  # mostly distinct
        k = rng.integers(0, 2 ** 62, n, dtype=np.int64)
    elif kind == 2:  # power law over a wide range
        k = np.floor(2.0 ** (rng.random(n) ** 3 * 40)).astype(np.int64)
    elif kind == 3:  # a skewed mix: one key for a random share, the rest spread
        k = rng.integers(0, max(2, n // 4), n, dtype=np.int64)
        k[rng.random(n) < rng.random()] = 12345
    else:  # small integers with duplicates
        k = rng.integers(0, max(2, n // 20), n, dtype=np.int64)
    return kind, k.astype(np.uint64)


def _params(rng):
    tmin = int(2 ** rng.integers(13, 17))
    tmax = int(2 ** rng.integers(int(np.log2(tmin)), 17))
    return S.default_params(
        n_light_log2=int(rng.integers(1, 11)),
        base_case=int(rng.choice([64, 256, 1000, 2048, 4096])),
        sample_mult=int(rng.choice([1, 20, 200, 800, 2000])),
        heavy_min=int(rng.integers(0, 8)),
        tile_min=tmin,
        tile_max=tmax,
        hash_mode=int(rng.integers(0, 2)),
    )


@pytest.mark.parametrize("case", range(CASES))
def test_random_shapes_and_parameters(case):
    rng = np.random.default_rng(1000 + case)
    n = int(10 ** rng.uniform(0, 5.6))
    kind, k = _keys(rng, n)
    p = _params(rng)
    v32 = rng.random() < 0.5
    v = np.arange(n, dtype=np.uint32 if v32 else np.uint64)
    _say(f"case {case}: n={n} keys={kind} nl={p.n_light_log2} alpha={p.base_case} c={p.sample_mult} "
         f"tau={p.heavy_min} tiles={p.tile_min}..{p.tile_max} hash={p.hash_mode} v32={v32}")

    ko, vo = S.semisort_equal(to_dev(k), to_dev(v), params=p)
    S.sync()
    assert_semisort_equal(k, v, to_host(ko, np.uint64), to_host(vo, v.dtype), mode=p.hash_mode,
                          ctx=f"case {case} semisort_=")

    ko, vo = S.semisort_less(to_dev(k), to_dev(v), params=p)
    S.sync()
    rk, rv = O.semisort_less(k, v)
    assert np.array_equal(to_host(ko, np.uint64), rk), f"case {case} semisort_< keys"
    assert np.array_equal(to_host(vo, v.dtype), rv), f"case {case} semisort_< values"

    vals = rng.integers(0, 2 ** 63, n, dtype=np.int64).astype(np.uint64)
    gk, gs = S.collect_reduce(to_dev(k), to_dev(vals), params=p)
    S.sync()
    gk, gs = to_host(gk, np.uint64), to_host(gs, np.uint64)
    o = np.argsort(gk, kind="stable")
    rk, rs = O.collect_reduce(k, vals)
    assert np.array_equal(gk[o], rk) and np.array_equal(gs[o], rs), f"case {case} collect-reduce"

    gk, gc = S.histogram(to_dev(k), params=p)
    S.sync()
    gk, gc = to_host(gk, np.uint64), to_host(gc, np.uint64)
    o = np.argsort(gk, kind="stable")
    rk, rc = O.histogram(k)
    assert np.array_equal(gk[o], rk) and np.array_equal(gc[o], rc), f"case {case} histogram"

    op = ("min", "max", "xor", "first", "last", "affine")[case % 6]
    if op == "affine":
        vals = vals | np.uint64(1 << 32)  # odd multipliers: every record changes its group's fold
    gk, gs = S.collect_reduce(to_dev(k), to_dev(vals), params=p, op=op)
    S.sync()
    gk, gs = to_host(gk, np.uint64), to_host(gs, np.uint64)
    o = np.argsort(gk, kind="stable")
    mk, ms = O.collect_reduce(k, vals, op=op)
    assert np.array_equal(gk[o], mk) and np.array_equal(gs[o], ms), f"case {case} collect-reduce {op}"

    gk, gc = S.histogram(to_dev(k), params=p, ordered=True)
    S.sync()
    assert np.array_equal(to_host(gk, np.uint64), rk), f"case {case} ordered histogram keys"
    assert np.array_equal(to_host(gc, np.uint64), rc), f"case {case} ordered histogram counts"
