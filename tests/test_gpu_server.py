"""The request server: every request served in a mix (several lanes at once,
small semisort_= requests packed into batched calls) gives exactly the result
the same request gives alone through the direct entry points, and those are
checked against the oracle."""
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


def _mix(count, seed):
    """Requests of mixed operations and sizes (log-uniform in [1e3, 3e5])."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        n = int(10 ** rng.uniform(3, 5.5))
        op = int(rng.integers(0, 4))
        name = ["exp1e-5_u32idx", "zipf0.8_1e8_u32idx", "zipf1.2_hashed", "uniform1e5_index"][int(rng.integers(0, 4))]
        k, v = I.np_workload(name, n, 100 + i)
        if op == S.OP_COLLECT_REDUCE or (op == S.OP_SEMISORT_EQUAL and i % 3 == 0):
            v = v.astype(np.uint64)
        reqs.append((op, k, v))
    return reqs


def _alone(op, kd, vd):
    if op == S.OP_SEMISORT_EQUAL:
        r = S.semisort_equal(kd, vd)
    elif op == S.OP_SEMISORT_LESS:
        r = S.semisort_less(kd, vd)
    elif op == S.OP_HISTOGRAM:
        r = S.histogram(kd)
    else:
        r = S.collect_reduce(kd, vd)
    S.sync()
    return r


def test_results_in_the_mix_equal_results_alone():
    reqs = _mix(60, 1)
    dev = []
    for op, k, v in reqs:
        dev.append((op, to_dev(k), to_dev(v)))
    torch.cuda.synchronize()  # the server's lanes do not wait for other streams
    alone = [_alone(op, kd, vd) for op, kd, vd in dev]
    srv = S.Server(lanes=3, pack_max_records=1 << 17, batch_records=1 << 20)
    try:
        outs, tickets = [], []
        for op, kd, vd in dev:
            oa = torch.empty_like(kd)
            ob = torch.empty_like(vd) if op in (S.OP_SEMISORT_EQUAL, S.OP_SEMISORT_LESS) else torch.empty_like(kd)
            outs.append((oa, ob))
            tickets.append(srv.submit(op, kd, vd if op != S.OP_HISTOGRAM else None, oa, ob))
        _say(f"case: 60 mixed requests submitted, {sum(1 for r in reqs if r[0] == 0)} semisort_=")
        srv.drain()
        st = srv.stats()
        assert st["completed"] == 60
        assert st["packed"] > 0, "no request was packed"
        for i, t in enumerate(tickets):
            done, status, lat, m = srv.poll(t)
            assert done and status == 0 and lat > 0
            op = dev[i][0]
            oa, ob = outs[i]
            if op in (S.OP_HISTOGRAM, S.OP_COLLECT_REDUCE):
                ak, av = alone[i]
                assert m == ak.numel(), f"request {i}: {m} groups, alone {ak.numel()}"
                assert torch.equal(oa[:m], ak) and torch.equal(ob[:m], av), f"request {i} differs from alone"
            else:
                ak, av = alone[i]
                assert torch.equal(oa, ak) and torch.equal(ob, av), f"request {i} (op {op}) differs from alone"
        # the alone results themselves against the oracle (a few of each kind)
        seen = set()
        for i, (op, k, v) in enumerate(reqs):
            if op in seen:
                continue
            seen.add(op)
            oa, ob = outs[i]
            if op == S.OP_SEMISORT_EQUAL:
                assert_semisort_equal(k, v, to_host(oa, np.uint64), to_host(ob, v.dtype), ctx=f"request {i}")
            elif op == S.OP_SEMISORT_LESS:
                rk, rv = O.semisort_less(k, v)
                assert np.array_equal(to_host(oa, np.uint64), rk) and np.array_equal(to_host(ob, v.dtype), rv)
            else:
                m = srv.poll(tickets[i])[3]
                gk, gv = to_host(oa[:m], np.uint64), to_host(ob[:m], np.uint64)
                o = np.argsort(gk, kind="stable")
                rk, rv = O.histogram(k) if op == S.OP_HISTOGRAM else O.collect_reduce(k, v)
                assert np.array_equal(gk[o], rk) and np.array_equal(gv[o], rv)
    finally:
        srv.close()


def test_small_budget_still_serves_everything():
    reqs = _mix(12, 2)
    dev = [(op, to_dev(k), to_dev(v)) for op, k, v in reqs]
    torch.cuda.synchronize()
    biggest = max(k.numel() for _, k, _ in dev)
    # room for about one request's workspace at a time: lanes take turns
    srv = S.Server(lanes=2, pack_max_records=0, hbm_budget=biggest * 28 + (100 << 20))
    try:
        tickets = []
        keep = []
        for op, kd, vd in dev:
            oa = torch.empty_like(kd)
            ob = torch.empty_like(vd) if op in (S.OP_SEMISORT_EQUAL, S.OP_SEMISORT_LESS) else torch.empty_like(kd)
            keep.append((oa, ob))
            tickets.append(srv.submit(op, kd, vd if op != S.OP_HISTOGRAM else None, oa, ob))
        srv.drain()
        for t in tickets:
            done, status, _, _ = srv.poll(t)
            assert done and status == 0
        assert srv.stats()["completed"] == 12
    finally:
        srv.close()


def test_rejects_bad_requests_and_tickets():
    srv = S.Server(lanes=1)
    try:
        k = torch.zeros(10, dtype=torch.int64, device="cuda")
        with pytest.raises(S.SemisortError):
            srv.submit(7, k, k, k, k)
        with pytest.raises(S.SemisortError):
            srv.poll(12345)
        t = srv.submit(S.OP_SEMISORT_EQUAL, k[:0], k[:0], k[:0], k[:0])
        assert srv.poll(t)[0]
    finally:
        srv.close()


def _digest(t, w1, w2):
    """Order-dependent 128-bit digest of an int64 tensor: two sums of the
    entries times fixed odd per-position weights, wrapping mod 2^64."""
    n = t.numel()
    return int((t * w1[:n]).sum()), int((t * w2[:n]).sum())


def test_full_trace_every_served_result_equals_its_alone_run():
    # The benchmark's served configuration: 20,000 requests of a Poisson
    # stream at 2000/s, sizes log-uniform in [1e4, 1e8], semisort_= /
    # histogram / collect-reduce over a device-resident pool, 200 GB budget,
    # four lanes.  Each output's digest is taken when the request completes
    # and compared with the digest of the same request run alone.
    import time
    R, P = 20_000, 10 ** 8
    tr = I.serving_trace(R, P, seed=8)
    pool = I.t_serving_pool(P, 8, "cuda")
    g = torch.Generator(device="cuda").manual_seed(99)
    w1 = torch.randint(-2 ** 62, 2 ** 62, (P,), device="cuda", generator=g) * 2 + 1
    w2 = torch.randint(-2 ** 62, 2 ** 62, (P,), device="cuda", generator=g) * 2 + 1
    torch.cuda.synchronize()
    opcode = {0: S.OP_SEMISORT_EQUAL, 1: S.OP_HISTOGRAM, 2: S.OP_COLLECT_REDUCE}

    def req(i):
        k, v = pool[int(tr["dists"][i])]
        a, n = int(tr["offs"][i]), int(tr["sizes"][i])
        return opcode[int(tr["ops"][i])], k[a:a + n], v[a:a + n]

    served = [None] * R
    srv = S.Server(lanes=4, hbm_budget=200 << 30)
    try:
        pending = {}
        out_bytes, cap = 0, 48 << 30

        def reap():
            nonlocal out_bytes
            for i in list(pending):
                t, oa, ob, nb = pending[i]
                done, st, _, m = srv.poll(t)
                if done:
                    assert st == 0, f"request {i} failed with {st}"
                    op = opcode[int(tr["ops"][i])]
                    if op != S.OP_SEMISORT_EQUAL:
                        oa, ob = oa[:m], ob[:m]
                    served[i] = (m, _digest(oa, w1, w2), _digest(ob, w1, w2))
                    out_bytes -= nb
                    del pending[i]

        base = srv.now()
        for i in range(R):
            op, k, v = req(i)
            nb = k.numel() * 16
            while out_bytes + nb > cap and pending:
                reap()
                time.sleep(0.0002)
            while srv.now() - base < tr["arrival"][i]:
                reap()
            oa, ob = torch.empty_like(k), torch.empty_like(k)
            t = srv.submit(op, k, v if op != S.OP_HISTOGRAM else None, oa, ob, arrival=base + tr["arrival"][i])
            pending[i] = (t, oa, ob, nb)
            out_bytes += nb
            if i % 2000 == 0:
                _say(f"served trace: {i} of {R} submitted")
        srv.drain()
        reap()
        assert not pending
        st = srv.stats()
        _say(f"served trace: {st['completed']} completed, {st['calls']} calls, {st['packed']} packed")
    finally:
        srv.close()
    ctx = S.context(0)
    for i in range(R):
        op, k, v = req(i)
        if op == S.OP_SEMISORT_EQUAL:
            oa, ob = S.semisort_equal(k, v, ctx=ctx)
            m = 0
        elif op == S.OP_HISTOGRAM:
            oa, ob = S.histogram(k, ctx=ctx)
            m = oa.numel()
        else:
            oa, ob = S.collect_reduce(k, v, ctx=ctx)
            m = oa.numel()
        ctx.sync()
        alone = (m, _digest(oa, w1, w2), _digest(ob, w1, w2))
        assert served[i] == alone, f"request {i} (op {op}, n {k.numel()}) differs from its alone run"
        if i % 2000 == 0:
            _say(f"alone runs: {i} of {R} match")
