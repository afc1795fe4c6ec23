"""Randomized GPU parity across the forms of the semisorts: key width (32,
64 or 128 bits), semisort_= or semisort_<, u32 or u64 values, out of place or
in place, the n-record temporary array or a pool of random size
(temp_records), and a random parameter set, each case compared with the
oracle: semisort_= in canonical form (Section 2.1: equal keys contiguous,
records of a key in input order), semisort_< element by element (the stable
sort by key).  The fixed tests pin each form; this one looks for
interactions between them."""
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

CASES = 30


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _words(rng, n):
    """u64 words with heavy keys, spread keys or both."""
    kind = int(rng.integers(0, 4))
    if kind == 0:
        w = rng.integers(0, int(rng.integers(1, 40)), n, dtype=np.uint64)
    elif kind == 1:
        w = rng.integers(0, 2 ** 63, n, dtype=np.uint64)
    elif kind == 2:
        w = np.floor(2.0 ** (rng.random(n) ** 3 * 40)).astype(np.uint64)
    else:
        w = rng.integers(0, max(2, n // 8), n, dtype=np.uint64)
        w[rng.random(n) < rng.random()] = np.uint64(987654321)
    return kind, w


def _keys(rng, n, kb):
    kind, w = _words(rng, n)
    if kb == 4:
        return kind, (w & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    if kb == 8:
        return kind, w
    # 128-bit keys: the second word is a function of the first (one key per
    # word), a few values (keys that share their low word), or random
    hk = int(rng.integers(0, 3))
    if hk == 0:
        hi = w * np.uint64(0x9E3779B97F4A7C15)
    elif hk == 1:
        hi = rng.integers(0, 3, n, dtype=np.uint64)
    else:
        hi = rng.integers(0, 2 ** 63, n, dtype=np.uint64)
    return kind * 10 + hk, np.stack([w, hi], axis=1)


def _params(rng, n):
    tmin = int(2 ** rng.integers(13, 17))
    tmax = int(2 ** rng.integers(int(np.log2(tmin)), 17))
    pool = 0 if rng.random() < 0.4 else int(rng.integers(1, max(2, n)))
    return S.default_params(
        n_light_log2=int(rng.integers(1, 11)),
        base_case=int(rng.choice([64, 256, 1000, 2048, 4096])),
        sample_mult=int(rng.choice([1, 20, 200, 800])),
        heavy_min=int(rng.integers(0, 8)),
        tile_min=tmin,
        tile_max=tmax,
        hash_mode=int(rng.integers(0, 2)),
        temp_records=pool,
    )


def _dev_keys(k):
    if k.ndim == 2:
        return torch.from_numpy(np.ascontiguousarray(k).view(np.int64)).cuda()
    return to_dev(k)


def _host_keys(t, k):
    if k.ndim == 2:
        return t.cpu().numpy().view(np.uint64)
    return to_host(t, k.dtype)


@pytest.mark.parametrize("case", range(CASES))
def test_random_widths_forms_and_parameters(case):
    rng = np.random.default_rng(5000 + case)
    n = int(10 ** rng.uniform(0, 5.6))
    kb = int(rng.choice([4, 8, 16]))
    kind, k = _keys(rng, n, kb)
    p = _params(rng, n)
    v = np.arange(n, dtype=np.uint32 if rng.random() < 0.5 else np.uint64)
    inplace = rng.random() < 0.3
    for less in (False, True):
        _say(f"case {case}: n={n} key_bytes={kb} keys={kind} less={less} in_place={inplace} "
             f"pool={p.temp_records} nl={p.n_light_log2} alpha={p.base_case} c={p.sample_mult} "
             f"tau={p.heavy_min} tiles={p.tile_min}..{p.tile_max} hash={p.hash_mode} v={v.dtype}")
        fn = S.semisort_less if less else S.semisort_equal
        kd, vd = _dev_keys(k), to_dev(v)
        if inplace:
            fn(kd, vd, kd, vd, params=p)
            ko, vo = kd, vd
        else:
            ko, vo = fn(kd, vd, params=p)
        S.sync()
        hk, hv = _host_keys(ko, k), to_host(vo, v.dtype)
        ctx = f"case {case} {'semisort_<' if less else 'semisort_='}"
        if kb == 16:
            rk, rv = O.semisort_equal_wide(k, v)  # the stable grouping, runs ordered by key
            if less:
                assert np.array_equal(hk, rk), f"{ctx}: keys differ from the oracle's sorted order"
                assert np.array_equal(hv, rv), f"{ctx}: values differ from the oracle's sorted order"
            else:
                bad, ck, cv = O.canonicalize_equal_wide(hk, hv)
                assert bad == -1, f"{ctx}: key at position {bad} starts a second run"
                assert np.array_equal(ck, rk) and np.array_equal(cv, rv), f"{ctx}: differs from the oracle"
        else:
            k64, h64 = k.astype(np.uint64), hk.astype(np.uint64)
            if less:
                rk, rv = O.semisort_less(k64, v)
                assert np.array_equal(h64, rk), f"{ctx}: keys differ from the oracle"
                assert np.array_equal(hv, rv), f"{ctx}: values differ from the oracle"
            else:
                assert_semisort_equal(k64, v, h64, hv, mode=p.hash_mode, ctx=ctx)
