"""GPU parity of semisort_= and semisort_< with 32-bit keys
(ss_semisort_equal_keys / ss_semisort_less_keys, key_bytes = 4): against the
oracle on the zero-extended keys (the library hashes a 32-bit key as its
zero-extended value, so the 64-bit oracle's canonical form applies), and bit
for bit against the 64-bit call on the zero-extended keys, which samples,
buckets and refines the same way.  Sizes span several subarrays with ragged
tails; edge cases: empty, single records, below the base case, in place,
all-equal keys, the extreme values, both value widths and both hashes."""
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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _k32_dev(k):
    return torch.from_numpy(np.ascontiguousarray(k, dtype=np.uint32).view(np.int32)).cuda()


def _run(less, k, v, params=None, inplace=False):
    kd, vd = _k32_dev(k), to_dev(v)
    if inplace:
        fn = S.semisort_less if less else S.semisort_equal
        fn(kd, vd, kd, vd, params=params)
        ko, vo = kd, vd
    else:
        ko, vo = (S.semisort_less if less else S.semisort_equal)(kd, vd, params=params)
    S.sync()
    return to_host(ko, np.uint32), to_host(vo, v.dtype)


def _check(less, k, v, params=None, ctx="", inplace=False):
    ko, vo = _run(less, k, v, params, inplace)
    k64 = k.astype(np.uint64)
    mode = params.hash_mode if params is not None else 0
    if less:
        rk, rv = O.semisort_less(k64, v)
        assert np.array_equal(ko.astype(np.uint64), rk), f"{ctx}: keys differ from the oracle"
        assert np.array_equal(vo, rv), f"{ctx}: values differ from the oracle"
    else:
        assert_semisort_equal(k64, v, ko.astype(np.uint64), vo, mode=mode, ctx=ctx)
    # the 64-bit call on the zero-extended keys gives the same output
    fn = S.semisort_less if less else S.semisort_equal
    wk, wv = fn(to_dev(k64), to_dev(v), params=params)
    S.sync()
    assert np.array_equal(to_host(wk, np.uint64), ko.astype(np.uint64)), f"{ctx}: keys differ from the 64-bit call"
    assert np.array_equal(to_host(wv, v.dtype), vo), f"{ctx}: values differ from the 64-bit call"


@pytest.mark.parametrize("name,n", [("zipf1.2_hashed_k32", 3_000_001), ("uniform1e9_k32", 2_500_003),
                                    ("exp1e-5_k32_u32idx", 1_700_001), ("zipf1.2_hashed_k32", 65_537)])
@pytest.mark.parametrize("less", [False, True])
def test_paper_distributions_32bit_keys(name, n, less):
    k, v = I.np_workload(name, n, 31)
    v = np.arange(n, dtype=v.dtype)  # record index: stability is visible
    _say(f"case: {'semisort_<' if less else 'semisort_='} {name} n={n}")
    _check(less, k, v, ctx=f"{name} n={n}")


@pytest.mark.parametrize("less", [False, True])
def test_edge_cases_32bit_keys(less):
    rng = np.random.default_rng(33)
    ext = np.array([0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF], dtype=np.uint32)
    cases = {
        "one record": np.array([7], dtype=np.uint32),
        "two records": np.array([0xFFFFFFFF, 0], dtype=np.uint32),
        "below the base case": rng.integers(0, 50, 3000, dtype=np.uint32),
        "extreme values": ext[rng.integers(0, ext.size, 200_003)],
        "all equal": np.full(150_001, 0xDEADBEEF, dtype=np.uint32),
        "all distinct": rng.permutation(np.arange(1_000_003, dtype=np.uint32)) * np.uint32(4099),
    }
    for name, k in cases.items():
        v = np.arange(k.size, dtype=np.uint64)
        _say(f"case: {name} n={k.size}")
        _check(less, k, v, ctx=name)
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    ko, _ = (S.semisort_less if less else S.semisort_equal)(e, torch.empty(0, dtype=torch.int64, device="cuda"))
    assert ko.numel() == 0


def test_in_place_identity_hash_u32_values_and_small_parameters():
    k, v = I.np_workload("zipf1.2_hashed_k32", 1_200_007, 34)
    v32 = np.arange(k.size, dtype=np.uint32)
    _check(False, k, v32, ctx="u32 values")
    _check(False, k, v32, ctx="in place", inplace=True)
    _check(False, k, v32, params=S.default_params(hash_mode="identity"), ctx="identity hash")
    p = S.default_params(n_light_log2=3, base_case=256, sample_mult=30, tile_min=8192, tile_max=8192)
    _check(False, k, v32, params=p, ctx="deep recursion")
    _check(True, k, v32, params=p, ctx="deep recursion, semisort_<")


def test_rejects_bad_key_widths():
    L = S.lib()
    ctx = S.context(0)
    k = torch.zeros(16, dtype=torch.int64, device="cuda")
    for kb in (0, 2, 16):
        st = L.ss_semisort_equal_keys(ctx.h, S._ptr(k), kb, S._ptr(k), 8, 16, S._ptr(torch.empty_like(k)),
                                      S._ptr(torch.empty_like(k)), None)
        assert st == S.SS_EINVAL
