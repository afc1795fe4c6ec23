"""GPU parity of the bounded-temporary form (ss_params.temp_records): when the
output is not the input, the first level writes every bucket to the output and
the levels below refine groups of subproblems through a pool instead of the
n-record temporary array T (Section 3.4 notes that T costs n extra records;
Section 6 names reducing that space as future work).  Sampling depends only on
the seed, the level and a subproblem's offset, so the result must equal the
call with T bit for bit; it is also checked against the oracle.  Cases: the
paper's distributions, pools from one subproblem per group to larger than the
input, both semisorts, 32- and 128-bit keys, u32 values, deep recursion,
batches of instances, and in-place calls (which keep T).  A fresh context
shows the workspace held: the pool, not T."""
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


def _dev_keys(k):
    if k.ndim == 2:
        return torch.from_numpy(np.ascontiguousarray(k).view(np.int64)).cuda()
    return to_dev(k)


def _both(fn, k, v, pool, **kw):
    kd, vd = _dev_keys(k), to_dev(v)
    a = fn(kd, vd, params=S.default_params(**kw))
    b = fn(kd, vd, params=S.default_params(temp_records=pool, **kw))
    S.sync()
    out = []
    for ko, vo in (a, b):
        out.append((ko.cpu().numpy().view(k.dtype), to_host(vo, v.dtype)))
    return out


@pytest.mark.parametrize("less", [False, True])
@pytest.mark.parametrize("name,n", [("zipf1.2_hashed", 2_000_003), ("uniform1e9", 1_500_007),
                                    ("uniform1e3", 1_000_003), ("exp1e-5_u32idx", 1_200_001)])
def test_pooled_equals_the_call_with_T(name, n, less):
    k, _ = I.np_workload(name, n, 81)
    v = np.arange(n, dtype=np.uint64)
    fn = S.semisort_less if less else S.semisort_equal
    for pool in (1, n // 16, n // 3, 2 * n):
        _say(f"case: {'semisort_<' if less else 'semisort_='} {name} n={n} pool={pool}")
        (ak, av), (bk, bv) = _both(fn, k, v, pool)
        assert np.array_equal(ak, bk) and np.array_equal(av, bv), f"{name} pool {pool}: differs from the call with T"
    if less:
        rk, rv = O.semisort_less(k, v)
        assert np.array_equal(bk, rk) and np.array_equal(bv, rv)
    else:
        assert_semisort_equal(k, v, bk, bv, ctx=f"{name} pooled")


def test_pooled_key_widths_values_and_deep_recursion():
    n = 1_000_003
    k32, _ = I.np_workload("zipf1.2_hashed_k32", n, 82)
    v32 = np.arange(n, dtype=np.uint32)
    for less in (False, True):
        _say(f"case: 32-bit keys pooled less={less}")
        fn = S.semisort_less if less else S.semisort_equal
        (ak, av), (bk, bv) = _both(fn, k32, v32, n // 10)
        assert np.array_equal(ak, bk) and np.array_equal(av, bv)
    k128, _ = I.np_workload("zipf1.2_hashed_k128", n, 83)
    v = np.arange(n, dtype=np.uint64)
    _say("case: 128-bit keys pooled")
    (ak, av), (bk, bv) = _both(S.semisort_equal, k128, v, n // 10)
    assert np.array_equal(ak, bk) and np.array_equal(av, bv)
    bad, ck, cv = O.canonicalize_equal_wide(bk, bv)
    rk, rv = O.semisort_equal_wide(k128, v)
    assert bad == -1 and np.array_equal(ck, rk) and np.array_equal(cv, rv)
    k, _ = I.np_workload("uniform1e9", n, 84)
    _say("case: deep recursion pooled")
    (ak, av), (bk, bv) = _both(S.semisort_equal, k, v, 5000, n_light_log2=3, base_case=256, sample_mult=30,
                               tile_min=8192, tile_max=8192)
    assert np.array_equal(ak, bk) and np.array_equal(av, bv)
    assert_semisort_equal(k, v, bk, bv, ctx="deep pooled")


def test_pooled_batches_and_in_place_calls():
    sizes = [5, 70_000, 1, 300_000, 4096, 900_001]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    n = int(offs[-1])
    k, _ = I.np_workload("zipf1.2_hashed", n, 85)
    v = np.arange(n, dtype=np.uint64)
    kd, vd = to_dev(k), to_dev(v)
    _say("case: pooled batch")
    ak, av = S.semisort_equal_batch(kd, vd, offs)
    bk, bv = S.semisort_equal_batch(kd, vd, offs, params=S.default_params(temp_records=50_000))
    S.sync()
    assert torch.equal(ak, bk) and torch.equal(av, bv)
    _say("case: in place with temp_records (keeps T)")
    ok, ov = S.semisort_equal(kd, vd)
    ik, iv = kd.clone(), vd.clone()
    S.semisort_equal(ik, iv, ik, iv, params=S.default_params(temp_records=50_000))
    S.sync()
    assert torch.equal(ik, ok) and torch.equal(iv, ov)
    assert_semisort_equal(k, v, to_host(ik, np.uint64), to_host(iv, np.uint64), ctx="in place")


def test_pooled_workspace_is_the_pool_not_T():
    n = 20_000_003
    k, v = I.t_workload("zipf1.2_hashed", n, 86, "cuda")
    held = {}
    for pool in (0, n // 16):
        ctx = S.Context(0)
        try:
            ko, vo = S.semisort_equal(k, v, params=S.default_params(temp_records=pool), ctx=ctx)
            ctx.sync()
            held[pool] = ctx.workspace_held()
        finally:
            ctx.close()
    _say(f"workspace held: with T {held[0]} bytes, pooled {held[n // 16]} bytes")
    # T alone is 16 bytes per record; the pooled form holds at most its pool
    # (or the longest subproblem) of those
    assert held[0] >= 16 * n
    assert held[n // 16] < held[0] - 12 * n


@pytest.mark.parametrize("name", ["zipf1.2_hashed", "uniform1e9", "zipf1.2_hashed_k32", "zipf1.2_hashed_k128"])
def test_in_place_equals_out_of_place(name):
    # In place, the first level must send every bucket to T (the output is
    # the array other blocks still read); the result is the out-of-place
    # call's, bit for bit, for both semisorts and every key width.
    n = 8_000_009
    k, _ = I.np_workload(name, n, 87)
    v = np.arange(n, dtype=np.uint64)
    for less in (False, True):
        fn = S.semisort_less if less else S.semisort_equal
        kd, vd = _dev_keys(k), to_dev(v)
        ok, ov = fn(kd, vd)
        ik, iv = kd.clone(), vd.clone()
        _say(f"case: in place {name} n={n} less={less}")
        fn(ik, iv, ik, iv)
        S.sync()
        assert torch.equal(ik, ok) and torch.equal(iv, ov), f"{name} less={less}: in place differs"
