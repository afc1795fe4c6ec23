"""GPU parity of semisort_= and semisort_< with 128-bit keys
(ss_semisort_equal_keys / ss_semisort_less_keys with key_bytes = 16, keys as
(low, high) word pairs) against the oracle's stable grouping of 128-bit keys:
semisort_= compared in canonical form (runs ordered by key), semisort_<
element by element (the oracle's grouping is the stable sort by key).
Section 2.1 takes keys of any type with an equality test; here the 64-bit
level hash of a key can collide, so the cases include keys that agree in one
word (the identity hash then collides on purpose): heavy keys sharing a low
word with light ones, many keys sharing a low word, keys sharing the high
word, and a heavy collision at a deeper level.  Sizes span several subarrays
with ragged tails; edge cases: empty, one and two records, below the base
case, all equal, in place, u32 values, deep recursion, bad arguments."""
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


def _k128_dev(k):
    return torch.from_numpy(np.ascontiguousarray(k, dtype=np.uint64).view(np.int64)).cuda()


def _check(k, v, params=None, ctx="", inplace=False):
    kd, vd = _k128_dev(k), to_dev(v)
    if inplace:
        S.semisort_equal(kd, vd, kd, vd, params=params)
        ko, vo = kd, vd
    else:
        ko, vo = S.semisort_equal(kd, vd, params=params)
    S.sync()
    hk = ko.cpu().numpy().view(np.uint64)
    hv = to_host(vo, v.dtype)
    rk, rv = O.semisort_equal_wide(k, v)
    bad, ck, cv = O.canonicalize_equal_wide(hk, hv)
    assert bad == -1, f"{ctx}: key at position {bad} starts a second run (equal keys not contiguous)"
    if not np.array_equal(ck, rk):
        i = int(np.nonzero((ck != rk).any(axis=1))[0][0])
        raise AssertionError(f"{ctx}: keys differ from the oracle at canonical position {i}")
    if not np.array_equal(cv, rv):
        i = int(np.nonzero(cv != rv)[0][0])
        raise AssertionError(f"{ctx}: values differ from the oracle at canonical position {i}")


@pytest.mark.parametrize("name,n", [("zipf1.2_hashed_k128", 3_000_001), ("uniform1e9_k128", 2_500_003),
                                    ("zipf1.2_hashed_k128", 65_537)])
@pytest.mark.parametrize("mode", ["mix64", "identity"])
def test_paper_distributions_128bit_keys(name, n, mode):
    k, v = I.np_workload(name, n, 51)
    v = np.arange(n, dtype=np.uint64)  # record index: stability is visible
    _say(f"case: semisort_= {name} n={n} hash={mode}")
    _check(k, v, params=S.default_params(hash_mode=mode), ctx=f"{name} n={n} {mode}")


def _collision_keys(n, seed):
    """Zipf-1.2 ranks whose keys share low words: rank r has low word r // 7
    (mixed) and high word r, so every low word is shared by up to seven keys,
    the heaviest keys among them; plus keys with one shared high word."""
    r = I.np_zipf(n, 1.2, 10 ** 6, seed, 0)
    lo = I.np_rehash(r // np.uint64(7))
    k = np.stack([lo, r], axis=1)
    return k


@pytest.mark.parametrize("mode", ["identity", "mix64"])
def test_keys_sharing_a_word(mode):
    p = S.default_params(hash_mode=mode)
    k = _collision_keys(2_000_003, 52)
    v = np.arange(k.shape[0], dtype=np.uint64)
    _say(f"case: shared low words, hash={mode}")
    _check(k, v, params=p, ctx=f"shared low words {mode}")
    # one low word for every key (the identity hash sees a single value until
    # the high word): a heavy key, medium keys and a light tail
    rng = np.random.default_rng(53)
    n = 1_500_007
    hi = np.where(rng.random(n) < 0.4, 7, rng.integers(0, 50_000, n)).astype(np.uint64)
    k = np.stack([np.full(n, 0xABCDEF, dtype=np.uint64), hi], axis=1)
    _say(f"case: one low word, hash={mode}")
    _check(k, v[:n], params=p, ctx=f"one low word {mode}")
    # one high word, low words from a skewed distribution
    k = np.stack([I.np_zipf(n, 1.1, 10 ** 5, 54, 0), np.full(n, 0x1234, dtype=np.uint64)], axis=1)
    _say(f"case: one high word, hash={mode}")
    _check(k, v[:n], params=p, ctx=f"one high word {mode}")


def test_deep_levels_and_small_parameters():
    # a small base case and few light bits per level force recursion past the
    # first 64 hash bits for keys sharing a low word
    k = _collision_keys(800_011, 55)
    v32 = np.arange(k.shape[0], dtype=np.uint32)
    p = S.default_params(n_light_log2=3, base_case=256, sample_mult=30, tile_min=8192, tile_max=8192,
                         hash_mode="identity")
    _say("case: deep recursion, identity hash, u32 values")
    _check(k, v32, params=p, ctx="deep identity")
    p = S.default_params(n_light_log2=3, base_case=256, sample_mult=30, tile_min=8192, tile_max=8192)
    _say("case: deep recursion, mixed hash, u32 values")
    _check(k, v32, params=p, ctx="deep mixed")


def test_edge_cases_128bit_keys():
    rng = np.random.default_rng(56)
    ext = np.array([[0, 0], [~0, ~0], [0, ~0], [~0, 0], [1, 0], [0, 1]], dtype=np.int64).view(np.uint64)
    cases = {
        "one record": np.array([[7, 9]], dtype=np.uint64),
        "two records": np.array([[1, 0], [0, 1]], dtype=np.uint64),
        "below the base case": np.stack([rng.integers(0, 5, 3000, dtype=np.uint64),
                                         rng.integers(0, 5, 3000, dtype=np.uint64)], axis=1),
        "extreme words": ext[rng.integers(0, ext.shape[0], 200_003)],
        "all equal": np.tile(np.array([[0xDEADBEEF, 0xFEEDFACE]], dtype=np.uint64), (150_001, 1)),
        "all distinct": np.stack([rng.permutation(np.arange(1_000_003, dtype=np.uint64)),
                                  np.zeros(1_000_003, dtype=np.uint64)], axis=1),
    }
    for name, k in cases.items():
        v = np.arange(k.shape[0], dtype=np.uint64)
        _say(f"case: {name} n={k.shape[0]}")
        _check(k, v, ctx=name)
        _check(k, v, params=S.default_params(hash_mode="identity"), ctx=name + " identity")
    k, _ = I.np_workload("zipf1.2_hashed_k128", 1_000_003, 57)
    v = np.arange(k.shape[0], dtype=np.uint64)
    _say("case: in place")
    _check(k, v, ctx="in place", inplace=True)
    e = torch.empty((0, 2), dtype=torch.int64, device="cuda")
    ko, _ = S.semisort_equal(e, torch.empty(0, dtype=torch.int64, device="cuda"))
    assert ko.shape == (0, 2)


def _check_less(k, v, params=None, ctx="", inplace=False):
    """semisort_< of 128-bit keys: exactly the oracle's stable sort by the key
    as a 128-bit unsigned number, element by element."""
    kd, vd = _k128_dev(k), to_dev(v)
    if inplace:
        S.semisort_less(kd, vd, kd, vd, params=params)
        ko, vo = kd, vd
    else:
        ko, vo = S.semisort_less(kd, vd, params=params)
    S.sync()
    hk = ko.cpu().numpy().view(np.uint64)
    hv = to_host(vo, v.dtype)
    rk, rv = O.semisort_equal_wide(k, v)
    if not np.array_equal(hk, rk):
        i = int(np.nonzero((hk != rk).any(axis=1))[0][0])
        raise AssertionError(f"{ctx}: key at position {i} differs from the oracle's sorted order")
    if not np.array_equal(hv, rv):
        i = int(np.nonzero(hv != rv)[0][0])
        raise AssertionError(f"{ctx}: value at position {i} differs from the oracle (stability or moves)")


@pytest.mark.parametrize("name,n", [("zipf1.2_hashed_k128", 3_000_001), ("uniform1e9_k128", 2_500_003),
                                    ("zipf1.2_hashed_k128", 65_537)])
def test_semisort_less_128bit_keys(name, n):
    k, _ = I.np_workload(name, n, 58)
    v = np.arange(n, dtype=np.uint64)
    _say(f"case: semisort_< {name} n={n}")
    _check_less(k, v, ctx=f"less {name} n={n}")


def test_semisort_less_128bit_keys_sharing_words_and_edges():
    k = _collision_keys(1_000_003, 59)
    v = np.arange(k.shape[0], dtype=np.uint64)
    for mode in ("mix64", "identity"):
        _say(f"case: semisort_< shared low words, hash={mode}")
        _check_less(k, v, params=S.default_params(hash_mode=mode), ctx=f"less shared {mode}")
    _say("case: semisort_< u32 values, in place, deep recursion")
    v32 = np.arange(k.shape[0], dtype=np.uint32)
    _check_less(k, v32, ctx="less u32 values")
    _check_less(k, v, ctx="less in place", inplace=True)
    p = S.default_params(n_light_log2=3, base_case=256, sample_mult=30, tile_min=8192, tile_max=8192)
    _check_less(k, v, params=p, ctx="less deep")
    rng = np.random.default_rng(60)
    ext = np.array([[0, 0], [~0, ~0], [0, ~0], [~0, 0], [1, 0], [0, 1]], dtype=np.int64).view(np.uint64)
    cases = {
        "one record": np.array([[7, 9]], dtype=np.uint64),
        "two records": np.array([[0, 1], [1, 0]], dtype=np.uint64),
        "below the base case": np.stack([rng.integers(0, 5, 3000, dtype=np.uint64),
                                         rng.integers(0, 5, 3000, dtype=np.uint64)], axis=1),
        "extreme words": ext[rng.integers(0, ext.shape[0], 200_003)],
        "all equal": np.tile(np.array([[0xDEADBEEF, 0xFEEDFACE]], dtype=np.uint64), (150_001, 1)),
        "all distinct": np.stack([rng.permutation(np.arange(600_001, dtype=np.uint64)),
                                  rng.permutation(np.arange(600_001, dtype=np.uint64)) % np.uint64(7)], axis=1),
    }
    for name, kk in cases.items():
        _say(f"case: semisort_< {name} n={kk.shape[0]}")
        _check_less(kk, np.arange(kk.shape[0], dtype=np.uint64), ctx=f"less {name}")


def test_rejects_what_128bit_keys_do_not_support():
    k = _k128_dev(np.zeros((64, 2), dtype=np.uint64))
    v = torch.zeros(64, dtype=torch.int64, device="cuda")
    # a key array at an 8-byte offset is not 16-byte aligned
    base = torch.zeros(129, dtype=torch.int64, device="cuda")
    with pytest.raises(S.SemisortError):
        S.semisort_equal(base[1:].view(64, 2), v)
    # outputs must be at least as large as the input
    with pytest.raises(ValueError):
        S.semisort_equal(k, v, torch.empty(64, dtype=torch.int64, device="cuda"), torch.empty_like(v))
