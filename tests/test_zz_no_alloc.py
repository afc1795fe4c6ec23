"""GPU tests of ss_semisort_equal_batch_noalloc, the batched semisort_= whose
workspace is the library's static scratch array (no allocation): its output
must equal, bit for bit, that of ss_semisort_equal_batch_capturable, the entry
point it is a variant of, on the same inputs -- on two calls in a row, the
second with a smaller input (the array keeps the first call's contents) --
and each instance must match the oracle.  Also: a batch whose worst case does
not fit is refused before anything runs, and a graph captured with no earlier
call replays correctly with new inputs."""
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


def _noalloc_vs_capturable(k, v, offs, ctx, params=None, oracle_instances=6, label=""):
    _say(f"case: {label} n={k.size} instances={len(offs) - 1} value bytes={v.dtype.itemsize}")
    kd, vd, od = to_dev(k), to_dev(v), _offs_dev(offs)
    ko = torch.empty_like(kd)
    vo = torch.empty_like(vd)
    S.semisort_equal_batch_noalloc(kd, vd, od, ko, vo, params=params, ctx=ctx)
    ctx.sync()
    rk, rv = S.semisort_equal_batch_capturable(kd, vd, od, params=params, ctx=ctx)
    ctx.sync()
    gk, gv = to_host(ko, np.uint64), to_host(vo, v.dtype)
    assert np.array_equal(gk, to_host(rk, np.uint64)), f"{label}: keys differ from the capturable call"
    assert np.array_equal(gv, to_host(rv, v.dtype)), f"{label}: values differ from the capturable call"
    step = max(1, (len(offs) - 1) // oracle_instances)
    mode = params.hash_mode if params is not None else 0
    for i in range(0, len(offs) - 1, step):
        a, b = int(offs[i]), int(offs[i + 1])
        assert_semisort_equal(k[a:b], v[a:b], gk[a:b], gv[a:b], mode=mode, ctx=f"{label} instance {i}")


def test_two_calls_in_a_row_second_smaller():
    ctx = S.Context(0)
    try:
        # first call: close to the largest batch the array holds (2^20 records)
        k, v, offs, _ = I.np_batch_workload(48, 1e3, 2e5, 1 << 20, 41)
        assert k.size <= 1 << 20
        _noalloc_vs_capturable(k, v, offs, ctx, label="first call")
        # second call, smaller, u32 values and other instances: must not see
        # anything the first call left in the array
        k2, v2, offs2, _ = I.np_batch_workload(17, 1e3, 6e4, 300_000, 42)
        v2 = (np.arange(k2.size, dtype=np.uint64) * 3).astype(np.uint32)
        _noalloc_vs_capturable(k2, v2, offs2, ctx, label="second call")
        # one instance of heavy keys, identity hash
        k3, v3 = I.np_workload("zipf1.2_hashed", 700_000, 43)
        p = S.default_params(hash_mode="identity")
        _noalloc_vs_capturable(k3, v3, np.array([0, k3.size], dtype=np.uint64), ctx, params=p, label="third call")
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_a_batch_that_does_not_fit_is_refused():
    ctx = S.Context(0)
    try:
        n = 1 << 21
        kd = torch.zeros(n, dtype=torch.int64, device="cuda")
        vd = torch.zeros(n, dtype=torch.int64, device="cuda")
        od = torch.tensor([0, n], dtype=torch.int64, device="cuda")
        _say("case: 2^21 records (more than the static array holds)")
        with pytest.raises(S.SemisortError) as e:
            S.semisort_equal_batch_noalloc(kd, vd, od, torch.empty_like(kd), torch.empty_like(vd), ctx=ctx)
        assert e.value.status == S.SS_EINVAL
        assert "static scratch" in str(e.value) or "workspace" in str(e.value)
        ctx.sync()
        # the context still works afterwards
        k, v, offs, _ = I.np_batch_workload(8, 1e3, 3e4, 100_000, 44)
        _noalloc_vs_capturable(k, v, offs, ctx, label="after the refusal")
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_graph_captured_without_an_earlier_call():
    ctx = S.Context(0)
    try:
        k0, v0, offs, _ = I.np_batch_workload(40, 1e3, 1e5, 800_000, 45)
        n = k0.size
        keys = torch.empty(n, dtype=torch.int64, device="cuda")
        vals = torch.empty(n, dtype=torch.int64, device="cuda")
        ko = torch.empty_like(keys)
        vo = torch.empty_like(vals)
        od = _offs_dev(offs)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        _say("case: capture with no earlier call")
        with torch.cuda.graph(g):
            S.semisort_equal_batch_noalloc(keys, vals, od, ko, vo, ctx=ctx)
        torch.cuda.synchronize()
        for r in range(3):
            kr = (k0 ^ np.uint64(0x2545F491 * (r + 1))) * np.uint64(0xD6E8FEB86659FD93)
            vr = v0 + np.uint64(r + 7)
            keys.copy_(to_dev(kr))
            vals.copy_(to_dev(vr))
            ko.fill_(-1)
            torch.cuda.synchronize()
            _say(f"case: replay {r}")
            g.replay()
            torch.cuda.synchronize()
            ctx.sync()
            rk, rv = S.semisort_equal_batch_capturable(keys, vals, od, ctx=ctx)
            ctx.sync()
            assert torch.equal(ko, rk), f"replay {r}: keys differ from the capturable call"
            assert torch.equal(vo, rv), f"replay {r}: values differ from the capturable call"
            _ = (keys.sum() + vals.sum()).item()
        del g
    finally:
        torch.cuda.synchronize()
        ctx.close()
