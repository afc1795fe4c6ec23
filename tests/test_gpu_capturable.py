"""GPU parity for the batched semisort_= sized on the device
(ss_semisort_equal_batch_capturable): every instance against the oracle and,
bit for bit, against the host-sized batched call (both sample the same
positions relative to each instance, so they give the same result); edge
cases of the instance list; the conditions it reports (too few levels, bad
offsets) forced from the host; and capture into a graph replayed several
times with new inputs, every replay checked."""
import sys

import numpy as np
import pytest

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


def _offs_dev(offs):
    return to_dev(np.asarray(offs, dtype=np.uint64))


def _check(k, v, offs, ko, vo, params=None, ctx=""):
    """Each instance against the oracle and the whole output against the
    host-sized batched call with the same parameters."""
    vd = v.dtype
    ko, vo = to_host(ko, np.uint64), to_host(vo, vd)
    for i in range(len(offs) - 1):
        a, b = int(offs[i]), int(offs[i + 1])
        mode = params.hash_mode if params is not None else 0
        assert_semisort_equal(k[a:b], v[a:b], ko[a:b], vo[a:b], mode=mode, ctx=f"{ctx} instance {i}")
    hk, hv = S.semisort_equal_batch(to_dev(k), to_dev(v), offs, params=params)
    S.sync()
    assert np.array_equal(to_host(hk, np.uint64), ko), f"{ctx}: keys differ from the host-sized batch"
    assert np.array_equal(to_host(hv, vd), vo), f"{ctx}: values differ from the host-sized batch"


def _run(k, v, offs, params=None, max_levels=6, ctx=""):
    _say(f"case: {ctx} n={k.size} instances={len(offs) - 1}")
    ko, vo = S.semisort_equal_batch_capturable(to_dev(k), to_dev(v), _offs_dev(offs), max_levels=max_levels,
                                               params=params)
    S.sync()
    _check(k, v, offs, ko, vo, params, ctx)


def test_batched_configuration_shape():
    k, v, offs, d = I.np_batch_workload(192, 1e3, 1e5, 3e6, 7)
    _run(k, v, offs, ctx="batch of 192")


def test_mixed_sizes_including_empty_and_single_records():
    rng = np.random.default_rng(31)
    sizes = [0, 1, 2, 100, 511, 512, 513, 1024, 1025, 2048, 2049, 4095, 4096, 10_000, 70_000, 3, 0, 1, 250_001]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    k = np.empty(int(offs[-1]), dtype=np.uint64)
    for i, sz in enumerate(sizes):
        a, b = int(offs[i]), int(offs[i + 1])
        k[a:b] = rng.integers(0, max(1, sz // 5), sz, dtype=np.int64).astype(np.uint64)
    v = np.arange(k.size, dtype=np.uint64)
    _run(k, v, offs, ctx="mixed sizes")


def test_all_small_and_one_large_instance():
    rng = np.random.default_rng(32)
    sizes = list(rng.integers(2, 4000, 300))
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    k = rng.integers(0, 50, int(offs[-1]), dtype=np.int64).astype(np.uint64)
    v = np.arange(k.size, dtype=np.uint64)
    _run(k, v, offs, ctx="all below alpha")
    k, v = I.np_workload("zipf1.2_hashed", 1_500_000, 3)
    _run(k, v, np.array([0, k.size], dtype=np.uint64), ctx="one zipf instance")
    k, v = I.np_workload("uniform1e9", 1_200_000, 4)
    _run(k, v, np.array([0, k.size], dtype=np.uint64), ctx="one uniform instance")


def test_u32_values_identity_hash_and_small_parameters():
    k, v, offs, d = I.np_batch_workload(64, 1e3, 5e4, 8e5, 9)
    v32 = (np.arange(k.size) * 7).astype(np.uint32)
    _run(k, v32, offs, ctx="u32 values")
    p = S.default_params(hash_mode="identity")
    _run(k, v, offs, params=p, ctx="identity hash")
    # deep recursion: few light buckets, small base case, small sample
    p = S.default_params(n_light_log2=2, base_case=256, sample_mult=20, tile_min=8192, tile_max=8192)
    _run(k, v, offs, params=p, max_levels=24, ctx="small parameters")


def test_in_place():
    k, v, offs, d = I.np_batch_workload(40, 1e3, 4e4, 4e5, 13)
    _say(f"case: in place n={k.size}")
    kd, vd = to_dev(k), to_dev(v)
    S.semisort_equal_batch_capturable(kd, vd, _offs_dev(offs), kd, vd)
    S.sync()
    _check(k, v, offs, kd, vd, ctx="in place")


def test_too_few_levels_is_reported_and_the_context_recovers():
    # 16 light buckets of ~125000 records each: a second level is needed
    k, v = I.np_workload("uniform1e9", 2_000_000, 5)
    offs = np.array([0, k.size], dtype=np.uint64)
    p = S.default_params(n_light_log2=4)
    _say("case: max_levels=1 on a two-level input")
    S.semisort_equal_batch_capturable(to_dev(k), to_dev(v), _offs_dev(offs), max_levels=1, params=p)
    with pytest.raises(S.SemisortError):
        S.sync()
    _run(k, v, offs, params=p, max_levels=2, ctx="after the reported condition")


def test_bad_offsets_are_reported():
    k = np.arange(10_000, dtype=np.uint64) % np.uint64(77)
    v = np.arange(10_000, dtype=np.uint64)
    _say("case: offsets that do not end at n")
    bad = np.array([0, 4000, 9000], dtype=np.uint64)  # n is 10000
    S.semisort_equal_batch_capturable(to_dev(k), to_dev(v), _offs_dev(bad))
    with pytest.raises(S.SemisortError):
        S.sync()
    _say("case: decreasing offsets")
    bad = np.array([0, 6000, 5000, 10_000], dtype=np.uint64)
    S.semisort_equal_batch_capturable(to_dev(k), to_dev(v), _offs_dev(bad))
    with pytest.raises(S.SemisortError):
        S.sync()


def test_rejected_arguments():
    k = torch.zeros(100, dtype=torch.int64, device="cuda")
    offs = torch.tensor([0, 100], dtype=torch.int64, device="cuda")
    with pytest.raises(S.SemisortError):
        S.semisort_equal_batch_capturable(k, k.clone(), offs, max_levels=0)
    with pytest.raises(S.SemisortError):
        S.semisort_equal_batch_capturable(k, k.clone(), offs, max_levels=65)


def test_graph_capture_and_replays_with_new_inputs():
    # A context of its own, so no other call grows the workspace the graph uses.
    ctx = S.Context(0)
    try:
        count, total = 96, 1_500_000
        k0, v0, offs, d = I.np_batch_workload(count, 1e3, 1e5, total, 21)
        n = k0.size
        keys = torch.empty(n, dtype=torch.int64, device="cuda")
        vals = torch.empty(n, dtype=torch.int64, device="cuda")
        ko = torch.empty_like(keys)
        vo = torch.empty_like(vals)
        od = _offs_dev(offs)
        keys.copy_(to_dev(k0))
        vals.copy_(to_dev(v0))
        _say("case: graph warm-up (sizes the workspace)")
        S.semisort_equal_batch_capturable(keys, vals, od, ko, vo, ctx=ctx)
        ctx.sync()
        _check(k0, v0, offs, ko, vo, ctx="warm-up")
        g = torch.cuda.CUDAGraph()
        _say("case: capture")
        with torch.cuda.graph(g):
            S.semisort_equal_batch_capturable(keys, vals, od, ko, vo, ctx=ctx)
        torch.cuda.synchronize()
        for r in range(4):
            # new keys for the same instance list each time (a bijection of
            # the old ones, so the groups stay but their hashes change), and
            # eager work on the stream between the replays
            kr = (k0 ^ np.uint64(0x5BD1E995 * (r + 1))) * np.uint64(0x9E3779B97F4A7C15)
            vr = v0 + np.uint64(r + 1)
            keys.copy_(to_dev(kr))
            vals.copy_(to_dev(vr))
            ko.fill_(-1)
            torch.cuda.synchronize()
            _say(f"case: replay {r}")
            g.replay()
            torch.cuda.synchronize()
            ctx.sync()
            _check(kr, vr, offs, ko, vo, ctx=f"replay {r}")
            _ = (keys.sum() + vals.sum()).item()
        del g
    finally:
        torch.cuda.synchronize()
        ctx.close()
