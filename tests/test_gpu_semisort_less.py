"""GPU parity for semisort_< : the result is unique (a stable sort by key), so
the HIP output must equal the oracle's element by element."""
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


def check_less(k, v, params=None, ctx=""):
    ko, vo = S.semisort_less(to_dev(k), to_dev(v), params=params)
    S.sync()  # waits and raises on a device-side error
    ko, vo = to_host(ko, np.uint64), to_host(vo, v.dtype)
    rk, rv = O.semisort_less(k, v)
    if not np.array_equal(ko, rk):
        i = int(np.nonzero(ko != rk)[0][0])
        raise AssertionError(f"{ctx}: keys differ at {i}: {ko[i]} vs {rk[i]}")
    if not np.array_equal(vo, rv):
        i = int(np.nonzero(vo != rv)[0][0])
        raise AssertionError(f"{ctx}: values differ at {i} (stability)")


@pytest.mark.parametrize("name,n", [("exp1e-5_u32idx", 2_000_003), ("zipf0.8_1e8_u32idx", 2_000_001),
                                    ("uniform1e9", 1_500_007), ("zipf1.2_hashed", 1_000_003),
                                    ("uniform1e5_index", 10 ** 6)])
def test_paper_distributions(name, n):
    k, v = I.np_workload(name, n, 31)
    _say(f"case: less {name} n={n}")
    check_less(k, v, ctx=name)


@pytest.mark.parametrize("n", [1, 2, 5, 64, 65, 4095, 4096, 4097, 70000, 300001])
def test_ragged_sizes(n):
    rng = np.random.default_rng(n + 1)
    k = rng.integers(0, max(2, n // 3), n, dtype=np.int64).astype(np.uint64)
    v = np.arange(n, dtype=np.uint64)
    _say(f"case: less ragged n={n}")
    check_less(k, v, ctx=f"n={n}")


def test_full_64_bit_keys_and_extremes():
    rng = np.random.default_rng(2)
    n = 400_000
    k = rng.integers(0, 2 ** 63, n, dtype=np.int64).astype(np.uint64) * np.uint64(2) + (rng.random(n) < 0.5).astype(np.uint64)
    k[::7] = np.uint64((1 << 64) - 1)
    k[::11] = np.uint64(0)
    v = np.arange(n, dtype=np.uint32)
    _say("case: less 64-bit keys")
    check_less(k, v, ctx="64-bit")


def test_all_equal():
    n = 100_000
    k = np.full(n, 42, dtype=np.uint64)
    v = np.arange(n, dtype=np.uint64)
    check_less(k, v, ctx="equal")


def test_deep_recursion_small_parameters():
    rng = np.random.default_rng(4)
    n = 200_000
    k = rng.integers(0, 50_000, n, dtype=np.int64).astype(np.uint64)
    v = np.arange(n, dtype=np.uint64)
    p = S.default_params(n_light_log2=2, base_case=64, sample_mult=30)
    _say("case: less deep")
    check_less(k, v, params=p, ctx="deep")


def test_batch_and_in_place():
    rng = np.random.default_rng(8)
    sizes = [3, 0, 5000, 1, 120_000, 4095]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    n = int(offs[-1])
    k = rng.integers(0, 1000, n, dtype=np.int64).astype(np.uint64)
    v = np.arange(n, dtype=np.uint32)
    kd, vd = to_dev(k), to_dev(v)
    _say("case: less batch in place")
    S.semisort_less_batch(kd, vd, offs, keys_out=kd, vals_out=vd)
    S.sync()  # waits and raises on a device-side error
    ko, vo = to_host(kd, np.uint64), to_host(vd, np.uint32)
    for i in range(len(sizes)):
        a, b = int(offs[i]), int(offs[i + 1])
        rk, rv = O.semisort_less(k[a:b], v[a:b])
        assert np.array_equal(ko[a:b], rk) and np.array_equal(vo[a:b], rv), f"instance {i}"


def test_boundary_table_cells():
    """The counting pass finds a key's bucket through a table of logarithmic
    cells of the key's offset from the smallest boundary: keys spread over
    all 64 octaves, keys in one narrow range, and two clusters 2^62 apart
    (most boundaries in a handful of cells, long searches inside a cell)."""
    rng = np.random.default_rng(9)
    n = 600_000
    cases = {
        "log-uniform": np.floor(2.0 ** (rng.random(n) * 63.99)).astype(np.uint64),
        "narrow": np.uint64(1 << 50) + rng.integers(0, 1_000_000, n, dtype=np.int64).astype(np.uint64),
        "two clusters": np.where(rng.random(n) < 0.5,
                                 rng.integers(0, 100_000, n, dtype=np.int64).astype(np.uint64),
                                 np.uint64(1 << 62) + rng.integers(0, 100_000, n, dtype=np.int64).astype(np.uint64)),
    }
    v = np.arange(n, dtype=np.uint64)
    for name, k in cases.items():
        _say(f"case: less cells {name}")
        check_less(k, v, ctx=name)
