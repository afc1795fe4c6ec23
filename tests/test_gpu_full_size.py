"""Parity at the full 10^9-record sizes, in the launch configuration the
benchmark times (default parameters, one call on the whole device-resident
input).  The oracle cannot process 10^9 records inside a test, so these check
properties that hold at any size -- the output is a permutation of the input,
equal keys are contiguous, records of a key keep their input order -- plus
sampled groups computed one by one by brute force (the input positions of one
key, in order, are exactly that group of a stable semisort)."""
import sys

import numpy as np
import pytest

from paper_2304_10078_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2304_10078_amd import semisort as S  # noqa: E402

N = 10 ** 9


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _indexed(name, seed):
    """Keys of a named workload with the record index as value (u64 or u32 as
    the workload's value width), so stability is visible in the output."""
    keys, vals = I.t_workload(name, N, seed, "cuda")
    idx = torch.arange(N, dtype=torch.int64, device="cuda")
    vals = idx if vals.dtype == torch.int64 else idx.to(torch.int32)
    return keys, vals


def _check_grouping(keys, ko, vo, ordered, samples=24, seed=0):
    vo64 = vo.to(torch.int64)
    # permutation: every input index appears once, and each record kept its key
    mark = torch.zeros(N, dtype=torch.bool, device="cuda")
    mark[vo64] = True
    assert bool(mark.all()), "output is not a permutation of the input"
    del mark
    assert bool(torch.equal(ko, keys[vo64])), "a record lost its key"
    same = ko[1:] == ko[:-1]
    if ordered:
        # ascending keys (as unsigned 64-bit words)
        a = ko[:-1] ^ torch.iinfo(torch.int64).min
        b = ko[1:] ^ torch.iinfo(torch.int64).min
        assert bool((a <= b).all()), "keys are not in ascending order"
    # contiguity: the keys that start runs are all different
    starts = torch.ones(N, dtype=torch.bool, device="cuda")
    starts[1:] = ~same
    run_keys = ko[starts]
    assert torch.unique(run_keys).numel() == run_keys.numel(), "a key occurs in two runs"
    # stability: inside a run the input indices increase
    assert bool(((vo64[1:] > vo64[:-1]) | ~same).all()), "records of a key lost their input order"
    # sampled groups against brute force
    g = torch.Generator(device="cpu").manual_seed(seed)
    picks = torch.randint(0, N, (samples,), generator=g).tolist()
    for p in picks:
        k = ko[p]
        want = torch.nonzero(keys == k).flatten()
        got = vo64[ko == k]
        assert torch.equal(got, want), f"group of key {int(k)} differs from the input positions"


def test_full_size_semisort_equal_zipf12_benchmark_configuration():
    keys, vals = _indexed("zipf1.2_hashed", 4)
    _say("case: semisort_= zipf1.2_hashed n=1e9 (benchmark configuration)")
    ko, vo = S.semisort_equal(keys, vals)
    S.sync()
    _check_grouping(keys, ko, vo, ordered=False)


def test_full_size_semisort_equal_uniform_1e9():
    keys, vals = _indexed("uniform1e9", 2)
    _say("case: semisort_= uniform[0,1e9) n=1e9")
    ko, vo = S.semisort_equal(keys, vals)
    S.sync()
    _check_grouping(keys, ko, vo, ordered=False, seed=1)


def test_full_size_semisort_less_exponential_u32_values():
    keys, vals = _indexed("exp1e-5_u32idx", 5)
    _say("case: semisort_< exp(1e-5) n=1e9, u32 values")
    ko, vo = S.semisort_less(keys, vals)
    S.sync()
    _check_grouping(keys, ko, vo, ordered=True, seed=2)


def test_full_size_collect_reduce_zipf12():
    keys, vals = I.t_workload("zipf1.2_hashed", N, 4, "cuda")
    _say("case: collect-reduce zipf1.2_hashed n=1e9")
    gk, gs = S.collect_reduce(keys, vals)
    S.sync()
    uk = torch.unique(keys)
    assert gk.numel() == uk.numel(), "number of groups differs from the distinct keys"
    assert torch.equal(torch.sort(gk).values, uk), "group keys differ from the distinct keys"
    # wrapping sums: the total is preserved mod 2^64 (int64 addition wraps the same way)
    assert int(gs.sum()) == int(vals.sum()), "sum of the group sums differs from the sum of the values"
    g = torch.Generator(device="cpu").manual_seed(3)
    for p in torch.randint(0, gk.numel(), (16,), generator=g).tolist():
        k = gk[p]
        assert int(gs[p]) == int(vals[keys == k].sum()), f"sum of key {int(k)} differs"
    # the heaviest key too
    top = uk[torch.argmax(torch.bincount(torch.searchsorted(uk, keys)))]
    p = int(torch.nonzero(gk == top).flatten()[0])
    assert int(gs[p]) == int(vals[keys == top].sum())


def test_full_size_histogram_zipf08():
    keys, _ = I.t_workload("zipf0.8_1e8_u32idx", N, 6, "cuda")
    _say("case: ordered histogram zipf0.8 over [1,1e8] n=1e9")
    gk, gc = S.histogram(keys, ordered=True)
    S.sync()
    # keys are positive, so torch's signed ascending order is the unsigned one
    uk, uc = torch.unique(keys, return_counts=True)
    assert gk.numel() == uk.numel()
    assert torch.equal(gk, uk) and torch.equal(gc, uc), "ordered histogram differs from the sorted distinct-key counts"


@pytest.mark.parametrize("kind", I.GRAPH_KINDS)
def test_full_size_graph_transpose(kind):
    # the benchmark's graphs: 1e9 edges over 5e7 vertices
    nv, ne = 50_000_000, N
    offs, cols = I.t_graph(kind, nv, ne, 5, "cuda")
    _say(f"case: transpose {kind} nv={nv} ne={ne}")
    oo, oc = S.transpose_csr(offs, cols)
    S.sync()
    # offsets: in-degree counts, accumulated
    deg = torch.bincount(cols.to(torch.int64), minlength=nv)
    assert int(oo[0]) == 0 and bool(torch.equal(oo[1:] - oo[:-1], deg)), "offsets differ from the in-degrees"
    del deg
    # sampled vertices: their in-neighbours are the sources of the edges into
    # them, in input order (the edge positions ascend, and so do their rows)
    g = torch.Generator(device="cpu").manual_seed(7)
    picks = torch.randint(0, ne, (8,), generator=g).tolist()
    for e in picks:
        v = int(cols[e]) & 0xFFFFFFFF
        pos = torch.nonzero(cols == v).flatten()
        src = torch.searchsorted(offs, pos, right=True) - 1
        got = oc[int(oo[v]):int(oo[v + 1])].to(torch.int64) & 0xFFFFFFFF
        assert torch.equal(got, src), f"in-neighbours of vertex {v} differ"
