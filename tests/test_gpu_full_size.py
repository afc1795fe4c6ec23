"""Parity at the full 10^9-record sizes, in the launch configuration the
benchmark times (default parameters, one call on the whole device-resident
input).  The oracle cannot process 10^9 records inside a test, so these check
complete properties that hold at any size and pin the result exactly:
- semisort: the output is a permutation of the input (values are record
  indices), every record kept its key, equal keys are contiguous, records of
  a key keep their input order (with ascending keys for semisort_<); a stable
  grouping is unique up to the order of its groups, so this is the whole
  definition (Section 2.1, stability as in Section 2.2);
- histogram and collect-reduce: EVERY group against a segment reduction of
  the input by key computed with library operations (unique + scatter),
  independent of the HIP path (Section 2.1, collect-reduce with the monoid);
- the in-order affine fold: every group against the oracle at 10^8 records,
  and sampled groups at 10^9 folded by the oracle one group at a time;
- the batch of 4096 instances: every instance by the same complete
  properties, and a sample of instances against the oracle;
plus sampled groups computed one by one by brute force."""
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
        # ascending keys (as unsigned words of the key's width)
        a = ko[:-1] ^ torch.iinfo(ko.dtype).min
        b = ko[1:] ^ torch.iinfo(ko.dtype).min
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


_SIGN = torch.iinfo(torch.int64).min


def _segment_reduce(keys, vals, op):
    """(distinct keys ascending as int64, per-key reduction): unique + scatter.
    Sums wrap mod 2^64 like int64 addition; min / max compare unsigned (the
    sign bit flipped maps unsigned order onto signed order)."""
    uk, inv = torch.unique(keys, return_inverse=True)
    m = uk.numel()
    if op == "count":
        r = torch.bincount(inv, minlength=m).to(torch.int64)
    elif op == "sum":
        r = torch.zeros(m, dtype=torch.int64, device=keys.device).index_add_(0, inv, vals)
    elif op in ("min", "max"):
        f = vals ^ _SIGN
        r = torch.empty(m, dtype=torch.int64, device=keys.device)
        r.scatter_reduce_(0, inv, f, "amin" if op == "min" else "amax", include_self=False)
        r ^= _SIGN
    else:
        raise ValueError(op)
    del inv
    return uk, r


def _check_reduce_complete(keys, vals, gk, gv, op, ordered=False):
    uk, want = _segment_reduce(keys, vals, op)
    assert gk.numel() == uk.numel(), f"{gk.numel()} groups, {uk.numel()} distinct keys"
    if ordered:
        # ascending as unsigned 64-bit words
        a, b = gk[:-1] ^ _SIGN, gk[1:] ^ _SIGN
        assert bool((a < b).all()), "ordered result keys are not strictly ascending"
    o = torch.argsort(gk)
    gk, gv = gk[o], gv[o]
    assert torch.equal(gk, uk), "group keys differ from the distinct keys"
    bad = torch.nonzero(gv != want).flatten()
    assert bad.numel() == 0, f"{op} of key {int(gk[bad[0]])} is {int(gv[bad[0]])}, expected {int(want[bad[0]])}"


@pytest.mark.parametrize("name,seed,op", [("zipf1.2_hashed", 4, "sum"), ("uniform1e9", 2, "sum"),
                                          ("uniform1e3", 3, "sum"), ("uniform1e9", 2, "min"),
                                          ("zipf1.2_hashed", 4, "max")])
def test_full_size_collect_reduce_every_group(name, seed, op):
    keys, vals = I.t_workload(name, N, seed, "cuda")
    _say(f"case: collect-reduce {op} {name} n=1e9")
    gk, gv = S.collect_reduce(keys, vals, op=op)
    S.sync()
    _check_reduce_complete(keys, vals, gk, gv, op)


def test_full_size_affine_fold_every_group_at_1e8():
    # every group against the oracle (the in-order fold needs the input
    # order, so no library reduction stands in for it)
    n = 10 ** 8
    keys, vals = I.t_workload("zipf1.2_hashed", n, 4, "cuda")
    vals = vals | (1 << 32)  # odd multipliers: invertible maps
    _say("case: collect-reduce affine zipf1.2_hashed n=1e8, every group against the oracle")
    gk, gv = S.collect_reduce(keys, vals, op="affine")
    S.sync()
    hk = keys.cpu().numpy().view(np.uint64)
    hv = vals.cpu().numpy().view(np.uint64)
    rk, rv = O.collect_reduce(hk, hv, op="affine")
    gk = gk.cpu().numpy().view(np.uint64)
    gv = gv.cpu().numpy().view(np.uint64)
    o = np.argsort(gk, kind="stable")
    assert np.array_equal(gk[o], rk), "group keys differ from the oracle"
    bad = np.nonzero(gv[o] != rv)[0]
    assert bad.size == 0, f"fold of key {rk[bad[0]]} differs from the oracle"


def test_full_size_affine_fold_sampled_groups():
    keys, vals = I.t_workload("zipf1.2_hashed", N, 4, "cuda")
    vals = vals | (1 << 32)
    _say("case: collect-reduce affine zipf1.2_hashed n=1e9, sampled groups")
    gk, gv = S.collect_reduce(keys, vals, op="affine")
    S.sync()
    assert gk.numel() == torch.unique(keys).numel()
    g = torch.Generator(device="cpu").manual_seed(5)
    picks = torch.randint(0, gk.numel(), (12,), generator=g).tolist()
    # and groups met at random record positions (heavier keys), below 5e6 records
    for p in torch.randint(0, N, (24,), generator=g).tolist():
        q = int(torch.nonzero(gk == keys[p]).flatten()[0])
        if len(picks) < 24 and int((keys == keys[p]).sum()) < 5_000_000:
            picks.append(q)
    for q in picks:
        k = gk[q]
        sel = torch.nonzero(keys == k).flatten()  # the group's records in input order
        gvk = vals[sel].cpu().numpy().view(np.uint64)
        rk, rv = O.collect_reduce(np.full(gvk.size, int(k) & (2 ** 64 - 1), dtype=np.uint64), gvk, op="affine")
        assert rk.size == 1 and int(rv[0]) == int(gv[q]) & (2 ** 64 - 1), f"fold of key {int(k)} differs"


def test_full_size_semisort_equal_uniform_1e3():
    keys, vals = _indexed("uniform1e3", 3)
    _say("case: semisort_= uniform[0,1e3) n=1e9")
    ko, vo = S.semisort_equal(keys, vals)
    S.sync()
    _check_grouping(keys, ko, vo, ordered=False, seed=4)


def test_full_size_semisort_less_zipf08_u32_values():
    keys, vals = _indexed("zipf0.8_1e8_u32idx", 6)
    _say("case: semisort_< zipf0.8 over [1,1e8] n=1e9, u32 values")
    ko, vo = S.semisort_less(keys, vals)
    S.sync()
    _check_grouping(keys, ko, vo, ordered=True, seed=5)


def test_full_size_semisort_equal_zipf12_32bit_keys():
    keys, vals = _indexed("zipf1.2_hashed_k32", 7)
    assert keys.dtype == torch.int32 and vals.dtype == torch.int32
    _say("case: semisort_= zipf1.2_hashed n=1e9, 32-bit keys and values")
    ko, vo = S.semisort_equal(keys, vals)
    S.sync()
    _check_grouping(keys, ko, vo, ordered=False, seed=7)


def test_full_size_semisort_less_exponential_32bit_keys():
    keys, vals = _indexed("exp1e-5_k32_u32idx", 8)
    assert keys.dtype == torch.int32 and vals.dtype == torch.int32
    _say("case: semisort_< exp(1e-5) n=1e9, 32-bit keys and values")
    ko, vo = S.semisort_less(keys, vals)
    S.sync()
    _check_grouping(keys, ko, vo, ordered=True, seed=8)


def test_full_size_semisort_equal_zipf12_128bit_keys():
    # 128-bit keys (low, high words): permutation, every record kept its key,
    # equal keys contiguous (the keys that start runs are distinct), stable,
    # and sampled groups by brute force.  Every gather is 1-D, one word at a
    # time: torch's row gather of an (n, 2) tensor returns zero rows once n
    # passes about 2^26 here.
    keys, vals = _indexed("zipf1.2_hashed_k128", 9)
    assert keys.shape == (N, 2)
    _say("case: semisort_= zipf1.2_hashed n=1e9, 128-bit keys, u64 values")
    ko, vo = S.semisort_equal(keys, vals)
    S.sync()
    mark = torch.zeros(N, dtype=torch.bool, device="cuda")
    mark[vo] = True
    assert bool(mark.all()), "output is not a permutation of the input"
    del mark
    same = None
    for w in (0, 1):
        kin = keys[:, w].contiguous()
        kout = ko[:, w].contiguous()
        assert bool(torch.equal(kout, kin[vo])), f"a record lost word {w} of its key"
        eq = kout[1:] == kout[:-1]
        same = eq if same is None else same & eq
        del kin, kout, eq
    starts = torch.ones(N, dtype=torch.bool, device="cuda")
    starts[1:] = ~same
    lo, hi = ko[:, 0].contiguous()[starts], ko[:, 1].contiguous()[starts]
    del starts
    # a key in two runs: two equal rows after a lexicographic sort (two
    # stable 1-D sorts, low word then high word)
    o = torch.sort(lo, stable=True).indices
    o = o[torch.sort(hi[o], stable=True).indices]
    slo, shi = lo[o], hi[o]
    assert not bool(((slo[1:] == slo[:-1]) & (shi[1:] == shi[:-1])).any()), "a key occurs in two runs"
    del lo, hi, o, slo, shi
    assert bool(((vo[1:] > vo[:-1]) | ~same).all()), "records of a key lost their input order"
    del same
    g = torch.Generator(device="cpu").manual_seed(9)
    for p in torch.randint(0, N, (12,), generator=g).tolist():
        k = ko[p]
        want = torch.nonzero((keys == k).all(dim=1)).flatten()
        got = vo[(ko == k).all(dim=1)]
        assert torch.equal(got, want), f"group of key {k.tolist()} differs from the input positions"


def test_full_size_semisort_less_zipf12_128bit_keys():
    # semisort_< of 128-bit keys: permutation, every record kept its key,
    # keys ascending as 128-bit unsigned numbers (high word, then low word),
    # records of a key in input order; 1-D gathers only
    keys, vals = _indexed("zipf1.2_hashed_k128", 9)
    _say("case: semisort_< zipf1.2_hashed n=1e9, 128-bit keys, u64 values")
    ko, vo = S.semisort_less(keys, vals)
    S.sync()
    mark = torch.zeros(N, dtype=torch.bool, device="cuda")
    mark[vo] = True
    assert bool(mark.all()), "output is not a permutation of the input"
    del mark
    for w in (0, 1):
        assert bool(torch.equal(ko[:, w].contiguous(), keys[:, w].contiguous()[vo])), f"a record lost word {w}"
    lo, hi = ko[:, 0].contiguous() ^ _SIGN, ko[:, 1].contiguous() ^ _SIGN  # unsigned order as signed
    up = (hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] >= lo[:-1]))
    assert bool(up.all()), "keys are not in ascending order"
    same = (hi[1:] == hi[:-1]) & (lo[1:] == lo[:-1])
    assert bool(((vo[1:] > vo[:-1]) | ~same).all()), "records of a key lost their input order"


def test_full_size_semisort_equal_pooled_uniform_1e9():
    # the bounded-temporary form: every level-1 subproblem refined through a
    # pool of n/16 records (uniform keys: all records reach level 1)
    keys, vals = _indexed("uniform1e9", 2)
    _say("case: semisort_= uniform[0,1e9) n=1e9 with a pool of n/16 records")
    ko, vo = S.semisort_equal(keys, vals, params=S.default_params(temp_records=N // 16))
    S.sync()
    _check_grouping(keys, ko, vo, ordered=False, seed=10)


def test_full_size_histogram_exponential():
    keys, _ = I.t_workload("exp1e-5_u32idx", N, 5, "cuda")
    _say("case: ordered histogram exp(1e-5) n=1e9")
    gk, gc = S.histogram(keys, ordered=True)
    S.sync()
    _check_reduce_complete(keys, None, gk, gc, "count", ordered=True)
    # keys are non-negative, so the signed ascending order is the unsigned one
    assert torch.equal(gk, torch.unique(keys))


def test_full_size_batch_every_instance():
    # the benchmark's batch: 4096 instances, 5e8 records, autotuned
    # parameters; values are the global record index
    keys, vals, offs, _ = I.t_batch_workload(4096, 1e3, 1e7, 5e8, 7, "cuda")
    n = keys.numel()
    ko, vo = torch.empty_like(keys), torch.empty_like(vals)
    best, _ = S.autotune_equal_batch(keys, vals, offs, ko, vo, reps=1)
    _say(f"case: batch of 4096 instances n={n}, tuned c={best.sample_mult} tau={best.heavy_min} "
         f"nl={best.n_light_log2} alpha={best.base_case} tmax={best.tile_max}")
    S.semisort_equal_batch(keys, vals, offs, ko, vo, params=best)
    S.sync()
    od = torch.from_numpy(np.asarray(offs, dtype=np.int64)).cuda()
    inst = torch.searchsorted(od, torch.arange(n, device="cuda"), right=True) - 1  # instance of each position
    # every record stays in its instance, once, with its key
    mark = torch.zeros(n, dtype=torch.bool, device="cuda")
    mark[vo] = True
    assert bool(mark.all()), "output is not a permutation of the input"
    del mark
    assert bool(torch.equal(inst[vo], inst)), "a record left its instance"
    assert bool(torch.equal(ko, keys[vo])), "a record lost its key"
    # contiguity per instance: (instance, key) starts one run only
    same = (ko[1:] == ko[:-1]) & (inst[1:] == inst[:-1])
    starts = torch.ones(n, dtype=torch.bool, device="cuda")
    starts[1:] = ~same
    rk, ri = ko[starts], inst[starts]
    o1 = torch.argsort(rk, stable=True)
    o = o1[torch.argsort(ri[o1], stable=True)]  # runs ordered by (instance, key)
    rk, ri = rk[o], ri[o]
    dup = (rk[1:] == rk[:-1]) & (ri[1:] == ri[:-1])
    assert not bool(dup.any()), "a key occurs in two runs of one instance"
    del rk, ri, o, o1, dup, starts
    assert bool(((vo[1:] > vo[:-1]) | ~same).all()), "records of a key lost their input order"
    # a sample of instances against the oracle, bit-exact after canonicalization
    o = [int(x) for x in offs]
    g = np.random.default_rng(12)
    for i in sorted(set(g.integers(0, 4096, 48).tolist())):
        a, b = o[i], o[i + 1]
        k = keys[a:b].cpu().numpy().view(np.uint64)
        v = vals[a:b].cpu().numpy().view(np.uint64)
        rk, rv = O.semisort_equal(k, v, best.hash_mode)
        bad, ck, cv = O.canonicalize_equal(ko[a:b].cpu().numpy().view(np.uint64),
                                           vo[a:b].cpu().numpy().view(np.uint64), best.hash_mode)
        assert bad == -1 and np.array_equal(ck, rk) and np.array_equal(cv, rv), f"instance {i} differs from the oracle"


def test_full_size_histogram_zipf08():
    keys, _ = I.t_workload("zipf0.8_1e8_u32idx", N, 6, "cuda")
    _say("case: ordered histogram zipf0.8 over [1,1e8] n=1e9")
    gk, gc = S.histogram(keys, ordered=True)
    S.sync()
    _check_reduce_complete(keys, None, gk, gc, "count", ordered=True)
    # keys are positive, so torch's signed ascending order is the unsigned one
    assert torch.equal(gk, torch.unique(keys))


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
