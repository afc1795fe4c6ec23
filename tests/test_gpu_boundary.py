"""GPU tests of the boundary's resource and batching calls:
- the workspace cap of ss_create: a context capped at the planning bound
  (ss_workspace_bytes) runs every operation and holds no more than the bound;
  a cap that is too small fails with SS_ENOMEM before anything runs, and the
  context still serves calls that fit;
- collect-reduce and histogram with m left on the device
  (ss_collect_reduce_async, ss_histogram_async): the same pairs, in the same
  order, as the calls that return m to the host;
- ss_batch over jobs of mixed operations, sizes and value widths: every job's
  output equals, bit for bit, the output of the single call, and its m; the
  single calls themselves are checked against the oracle elsewhere, and a
  sample here;
- ss_batch refuses overlapping and malformed jobs before touching anything;
- the server packs small requests of every operation into one call and never
  reserves more than its budget."""
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


def _run_op(op, kd, vd, ctx):
    """The single call of op; returns host arrays (keys, second output)."""
    if op == S.OP_SEMISORT_EQUAL:
        a, b = S.semisort_equal(kd, vd, ctx=ctx)
    elif op == S.OP_SEMISORT_LESS:
        a, b = S.semisort_less(kd, vd, ctx=ctx)
    elif op == S.OP_HISTOGRAM:
        a, b = S.histogram(kd, ctx=ctx)
    else:
        a, b = S.collect_reduce(kd, vd, ctx=ctx)
    ctx.sync()
    vt = np.uint32 if b.dtype == torch.int32 else np.uint64
    return to_host(a, np.uint64), to_host(b, vt)


@pytest.mark.parametrize("op", [S.OP_SEMISORT_EQUAL, S.OP_SEMISORT_LESS, S.OP_HISTOGRAM, S.OP_COLLECT_REDUCE])
def test_capped_context_runs_within_the_planning_bound(op):
    n = 3_000_000
    k, v = I.np_workload("zipf1.2_hashed", n, 51)
    if op == S.OP_SEMISORT_LESS:
        k, v = I.np_workload("exp1e-5_u32idx", n, 52)
    kd, vd = to_dev(k), to_dev(v)
    vb = 4 if v.dtype == np.uint32 else 8
    bound = S.workspace_bound(op, n, vb if op in (S.OP_SEMISORT_EQUAL, S.OP_SEMISORT_LESS) else 8)
    _say(f"case: op {op} n={n} cap=bound={bound}")
    ctx = S.Context(0, workspace_cap=bound)
    try:
        got = _run_op(op, kd, vd, ctx)
        held = ctx.workspace_held()
        assert held <= bound, (held, bound)
        free = S.Context(0)
        try:
            want = _run_op(op, kd, vd, free)
        finally:
            free.close()
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    finally:
        ctx.close()


def test_a_cap_too_small_fails_with_enomem_and_the_context_recovers():
    n = 2_000_000
    k, v = I.np_workload("uniform1e9", n, 53)
    kd, vd = to_dev(k), to_dev(v)
    ctx = S.Context(0, workspace_cap=4 << 20)
    try:
        _say("case: semisort_= of 2e6 records under a 4 MiB cap")
        ko = torch.full_like(kd, 7)
        with pytest.raises(S.SemisortError) as e:
            S.semisort_equal(kd, vd, ko, torch.empty_like(vd), ctx=ctx)
        assert e.value.status == S.SS_ENOMEM
        assert ctx.workspace_held() <= 4 << 20
        with pytest.raises(S.SemisortError) as e:
            S.collect_reduce(kd, vd, ctx=ctx)
        assert e.value.status == S.SS_ENOMEM
        # a call that fits still runs, correctly
        ks, vs = k[:3000], v[:3000]
        a, b = S.semisort_equal(to_dev(ks), to_dev(vs), ctx=ctx)
        ctx.sync()
        assert_semisort_equal(ks, vs, to_host(a, np.uint64), to_host(b, np.uint64), ctx="after ENOMEM")
        assert ctx.workspace_held() <= 4 << 20
    finally:
        ctx.close()


@pytest.mark.parametrize("op,ordered", [("sum", 0), ("min", 0), ("xor", 1), ("first", 0), ("last", 1),
                                        ("affine", 0), ("sum", 1)])
def test_collect_reduce_with_m_on_the_device(op, ordered):
    n = 1_200_000
    k, _ = I.np_workload("zipf0.8_1e8_u32idx", n, 54)
    rng = np.random.default_rng(55)
    v = rng.integers(0, 2 ** 63, n, dtype=np.int64).astype(np.uint64) * np.uint64(2) + np.uint64(1)
    kd, vd = to_dev(k), to_dev(v)
    _say(f"case: collect-reduce {op} ordered={ordered} with m on the device")
    ok, ov = torch.full_like(kd, -1), torch.full_like(kd, -1)
    dm = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    S.collect_reduce_async(kd, vd, dm, ok, ov, op=op, ordered=bool(ordered))
    S.sync()
    m = int(dm.item())
    rk, rv = S.collect_reduce(kd, vd, op=op, ordered=bool(ordered))
    S.sync()
    assert m == rk.numel()
    assert torch.equal(ok[:m], rk) and torch.equal(ov[:m], rv)


@pytest.mark.parametrize("ordered", [0, 1])
def test_histogram_with_m_on_the_device(ordered):
    n = 900_000
    k, _ = I.np_workload("exp1e-5_u32idx", n, 56)
    kd = to_dev(k)
    _say(f"case: histogram ordered={ordered} with m on the device")
    ok, oc = torch.empty_like(kd), torch.empty_like(kd)
    dm = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    S.histogram_async(kd, dm, ok, oc, ordered=bool(ordered))
    S.sync()
    m = int(dm.item())
    rk, rc = S.histogram(kd, ordered=bool(ordered))
    S.sync()
    assert m == rk.numel()
    assert torch.equal(ok[:m], rk) and torch.equal(oc[:m], rc)
    # and n = 0 writes m = 0
    S.histogram_async(kd[:0], dm, ok, oc)
    S.sync()
    assert int(dm.item()) == 0


def _mixed_jobs(seed, count, big=0):
    rng = np.random.default_rng(seed)
    names = ["exp1e-5_u32idx", "zipf0.8_1e8_u32idx", "zipf1.2_hashed", "uniform1e5_index", "uniform1e3"]
    jobs = []
    sizes = [0, 1, 2, 100, 4095, 4096, 4097] + [int(10 ** rng.uniform(2, 5.7)) for _ in range(count)]
    if big:
        sizes.append(big)
    for i, n in enumerate(sizes):
        op = i % 4
        k, v = I.np_workload(names[i % len(names)], max(n, 1), 500 + i)
        k, v = k[:n], v[:n]
        if op in (S.OP_HISTOGRAM, S.OP_COLLECT_REDUCE):
            v = v.astype(np.uint64)
        elif i % 3 == 0:
            v = v.astype(np.uint64)
        else:
            v = v.astype(np.uint32)
        jobs.append((op, k, v))
    return jobs


def _batch_vs_single(jobs, params=None):
    dev = []
    for op, k, v in jobs:
        kd, vd = to_dev(k), to_dev(v)
        oa = torch.full_like(kd, -1)
        ob = torch.full_like(vd if op < 2 else kd, -1)
        dm = torch.full((1,), -1, dtype=torch.int64, device="cuda") if op >= 2 else None
        dev.append((op, kd, vd if op != S.OP_HISTOGRAM else None, oa, ob, dm))
    torch.cuda.synchronize()
    _say(f"case: batch of {len(jobs)} jobs, {sum(k.size for _, k, _ in jobs)} records")
    S.batch(dev, params=params)
    S.sync()
    for i, ((op, k, v), (_, kd, vd, oa, ob, dm)) in enumerate(zip(jobs, dev)):
        n = k.size
        if op < 2:
            ra, rb = (S.semisort_equal if op == 0 else S.semisort_less)(kd, vd, params=params)
            S.sync()
            assert torch.equal(oa, ra), f"job {i} (op {op}, n {n}): keys differ from the single call"
            assert torch.equal(ob, rb), f"job {i} (op {op}, n {n}): values differ from the single call"
        else:
            m = int(dm.item())
            ra, rb = S.histogram(kd, params=params) if op == 2 else S.collect_reduce(kd, vd, params=params)
            S.sync()
            assert m == ra.numel(), f"job {i} (op {op}, n {n}): m {m} != {ra.numel()}"
            assert torch.equal(oa[:m], ra) and torch.equal(ob[:m], rb), f"job {i} (op {op}): pairs differ"
    return dev


def test_batch_of_mixed_jobs_equals_the_single_calls():
    jobs = _mixed_jobs(57, 60)
    dev = _batch_vs_single(jobs)
    # a sample against the oracle
    for i in (8, 9, 10, 11, 20, 33):
        op, k, v = jobs[i]
        _, _, _, oa, ob, dm = dev[i]
        if op == 0:
            assert_semisort_equal(k, v, to_host(oa, np.uint64), to_host(ob, v.dtype), ctx=f"job {i}")
        elif op == 1:
            rk, rv = O.semisort_less(k, v)
            assert np.array_equal(to_host(oa, np.uint64), rk) and np.array_equal(to_host(ob, v.dtype), rv)
        else:
            m = int(dm.item())
            gk, gv = to_host(oa[:m], np.uint64), to_host(ob[:m], np.uint64)
            o = np.argsort(gk, kind="stable")
            rk, rv = O.histogram(k) if op == 2 else O.collect_reduce(k, v)
            assert np.array_equal(gk[o], rk) and np.array_equal(gv[o], rv), f"job {i}"


def test_batch_with_a_job_above_the_packing_limit_and_identity_hash():
    jobs = _mixed_jobs(58, 12, big=(1 << 22) + 12345)
    _batch_vs_single(jobs)
    _batch_vs_single(_mixed_jobs(59, 16), params=S.default_params(hash_mode="identity"))


def test_batch_refuses_bad_jobs_before_running():
    n = 5000
    a = torch.arange(n, dtype=torch.int64, device="cuda")
    b = torch.arange(n, dtype=torch.int64, device="cuda")
    o1, o2 = torch.full_like(a, 7), torch.full_like(a, 7)
    dm = torch.zeros(2, dtype=torch.int64, device="cuda")
    good = (S.OP_SEMISORT_EQUAL, a, b, o1, o2, None)
    cases = {
        "outputs of two jobs overlap": [good, (S.OP_SEMISORT_EQUAL, a, b, o1[10:], torch.empty_like(a), None)],
        "output overlaps another job's input": [good, (S.OP_SEMISORT_LESS, o1, b, torch.empty_like(a),
                                                       torch.empty_like(a), None)],
        "in place": [(S.OP_SEMISORT_EQUAL, a, b, a, b, None)],
        "reduction without d_m": [(S.OP_HISTOGRAM, a, None, o1, o2, None)],
        "shared d_m": [(S.OP_HISTOGRAM, a, None, o1, o2, dm[:1]),
                       (S.OP_COLLECT_REDUCE, a, b, torch.empty_like(a), torch.empty_like(a), dm[:1])],
        "unknown op": [(9, a, b, o1, o2, None)],
    }
    for name, jobs in cases.items():
        _say(f"case: batch with {name}")
        with pytest.raises(S.SemisortError) as e:
            S.batch(jobs)
        assert e.value.status == S.SS_EINVAL, name
    S.sync()
    assert bool((o1 == 7).all()) and bool((o2 == 7).all()), "a refused batch wrote an output"


def test_server_packs_every_operation_within_its_budget():
    rng = np.random.default_rng(60)
    reqs = []
    for i in range(48):
        n = int(10 ** rng.uniform(3, 5))
        op = i % 4
        k, v = I.np_workload("zipf0.8_1e8_u32idx", n, 600 + i)
        v = v.astype(np.uint64)
        reqs.append((op, to_dev(k), to_dev(v)))
    torch.cuda.synchronize()
    budget = 1 << 30
    srv = S.Server(lanes=2, hbm_budget=budget)
    try:
        # a lane busy with a large request lets the small ones queue up
        kb, vb = I.np_workload("uniform1e9", 4_000_000, 61)
        kbd, vbd = to_dev(kb), to_dev(vb)
        outs = [(torch.empty_like(kbd), torch.empty_like(vbd))]
        tickets = [srv.submit(S.OP_SEMISORT_EQUAL, kbd, vbd, *outs[0])]
        for op, kd, vd in reqs:
            oa, ob = torch.empty_like(kd), torch.empty_like(vd)
            outs.append((oa, ob))
            tickets.append(srv.submit(op, kd, vd if op != S.OP_HISTOGRAM else None, oa, ob))
        srv.drain()
        st = srv.stats()
        _say(f"server stats: {st}")
        assert st["completed"] == len(tickets)
        assert st["peak_reserved"] <= budget
        assert st["packed"] > 0 and st["calls"] < len(tickets)
        for i, (op, kd, vd) in enumerate(reqs):
            done, status, _, m = srv.poll(tickets[i + 1])
            assert done and status == 0
            oa, ob = outs[i + 1]
            ra, rb = _run_op(op, kd, vd, S.context(0))
            if op < 2:
                assert np.array_equal(to_host(oa, np.uint64), ra) and np.array_equal(to_host(ob, np.uint64), rb)
            else:
                assert m == ra.size
                assert np.array_equal(to_host(oa[:m], np.uint64), ra) and np.array_equal(to_host(ob[:m], np.uint64),
                                                                                        rb)
    finally:
        srv.close()
