"""Pins for the CPU oracle: it is checked here against the problem definitions
(Section 2.1), stability (Section 2.2), brute force on tiny inputs, library
routines and closed forms -- never against itself."""
import itertools
import math
from collections import Counter

import numpy as np
import pytest

import oracle as O

ALPHABET = [0, 1, 1 << 63, (1 << 64) - 1]
MOD = 1 << 64


def _all_sequences(max_len):
    for n in range(max_len + 1):
        for seq in itertools.product(ALPHABET, repeat=n):
            yield list(seq)


# ---------------------------------------------------------------- hash pins


def _inv_xorshift(y, s):
    x = y
    for _ in range(64 // s + 1):
        x = y ^ (x >> s)
    return x


def test_hash_is_a_bijection_with_the_published_inverse():
    # Invert the finalizer step by step with modular inverses of its two
    # multipliers; a wrong constant or shift anywhere breaks the round trip.
    c1 = 0xFF51AFD7ED558CCD
    c2 = 0xC4CEB9FE1A85EC53
    i1, i2 = pow(c1, -1, MOD), pow(c2, -1, MOD)
    rng = np.random.default_rng(1)
    xs = [0, 1, 2, (1 << 64) - 1, 1 << 63] + [int(v) for v in rng.integers(0, 2 ** 63, 200, dtype=np.int64)]
    for x in xs:
        y = O.hash64(x)
        z = _inv_xorshift(y, 33)
        z = (z * i2) % MOD
        z = _inv_xorshift(z, 33)
        z = (z * i1) % MOD
        z = _inv_xorshift(z, 33)
        assert z == x
    assert O.hash64(0) == 0
    assert O.hash64(12345, O.HASH_IDENTITY) == 12345


def test_hash_low_bits_spread_consecutive_keys():
    # The light bucket id uses low hash bits; consecutive integers must land
    # in all 1024 buckets about evenly (chi-square, 1023 dof).
    h = np.array([O.hash64(i) for i in range(1 << 16)], dtype=np.uint64)
    counts = np.bincount((h & np.uint64(1023)).astype(np.int64), minlength=1024)
    exp = (1 << 16) / 1024
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 1023 + 6 * math.sqrt(2 * 1023)


# ------------------------------------------------ definitions, exhaustively


def _check_semisort_equal(keys, ko, vo):
    n = len(keys)
    vo = [int(v) for v in vo]
    ko = [int(k) for k in ko]
    assert sorted(vo) == list(range(n))  # a permutation of the records
    assert all(ko[p] == keys[vo[p]] for p in range(n))  # records moved whole
    seen = set()
    for p in range(n):  # equal keys contiguous
        if p == 0 or ko[p] != ko[p - 1]:
            assert ko[p] not in seen
            seen.add(ko[p])
    for p in range(1, n):  # stable: input order kept inside a group
        if ko[p] == ko[p - 1]:
            assert vo[p] > vo[p - 1]


def test_semisort_equal_exhaustive_tiny():
    count = 0
    for keys in _all_sequences(7):
        n = len(keys)
        k = np.array(keys, dtype=np.uint64)
        v = np.arange(n, dtype=np.uint64)
        ko, vo = O.semisort_equal(k, v)
        _check_semisort_equal(keys, ko, vo)
        # canonical group order: ascending hash of the group's key
        firsts = [int(ko[p]) for p in range(n) if p == 0 or ko[p] != ko[p - 1]]
        hs = [O.hash64(x) for x in firsts]
        assert hs == sorted(hs)
        count += 1
    assert count == sum(4 ** i for i in range(8))


def test_semisort_less_is_pythons_stable_sort():
    for keys in _all_sequences(6):
        n = len(keys)
        k = np.array(keys, dtype=np.uint64)
        v = np.arange(n, dtype=np.uint32)
        ko, vo = O.semisort_less(k, v)
        order = sorted(range(n), key=lambda i: keys[i])  # Python's sort is stable
        assert [int(x) for x in vo] == order
        assert [int(x) for x in ko] == [keys[i] for i in order]


def test_histogram_and_collect_reduce_brute_force():
    rng = np.random.default_rng(7)
    for keys in _all_sequences(5):
        n = len(keys)
        # values near 2^64 force wrap-around
        vals = [int(x) for x in rng.integers(0, 2 ** 63, n, dtype=np.int64)]
        vals = [(MOD - 1 - v) if i % 2 else v for i, v in enumerate(vals)]
        k = np.array(keys, dtype=np.uint64)
        v = np.array(vals, dtype=np.uint64)
        hk, hc = O.histogram(k)
        ck, cs = O.collect_reduce(k, v)
        uniq = sorted(set(keys))
        assert [int(x) for x in hk] == uniq and [int(x) for x in ck] == uniq
        for j, u in enumerate(uniq):
            assert int(hc[j]) == sum(1 for x in keys if x == u)
            assert int(cs[j]) == sum(vals[i] for i in range(n) if keys[i] == u) % MOD
        assert int(hc.sum()) == n


def test_collect_reduce_monoids_brute_force():
    # every key sequence of length <= 5 over 3 keys; per key the fold of its
    # values by Python's own min / max / ^ (the monoids' definitions)
    rng = np.random.default_rng(17)
    ops = {"min": min, "max": max, "xor": lambda a, b: a ^ b}
    for keys in _all_sequences(5):
        n = len(keys)
        vals = [int(x) for x in rng.integers(0, 2 ** 63, n, dtype=np.int64)]
        vals = [(MOD - 1 - v) if i % 3 == 1 else v for i, v in enumerate(vals)]  # top bit set too
        k = np.array(keys, dtype=np.uint64)
        v = np.array(vals, dtype=np.uint64)
        uniq = sorted(set(keys))
        for name, f in ops.items():
            ck, cv = O.collect_reduce(k, v, op=name)
            assert [int(x) for x in ck] == uniq
            for j, u in enumerate(uniq):
                group = [vals[i] for i in range(n) if keys[i] == u]
                acc = group[0]
                for x in group[1:]:
                    acc = f(acc, x)
                assert int(cv[j]) == acc, (name, keys, u)


def test_collect_reduce_monoids_match_numpy_segment_reductions():
    # the same folds by numpy's ufunc.reduceat over the key-sorted values
    rng = np.random.default_rng(29)
    for n, M in [(1, 1), (2000, 7), (30000, 5000)]:
        k = rng.integers(0, M, n, dtype=np.int64).astype(np.uint64)
        v = rng.integers(0, 2 ** 63, n, dtype=np.int64).astype(np.uint64) * np.uint64(3)
        o = np.argsort(k, kind="stable")
        ks, vs = k[o], v[o]
        starts = np.flatnonzero(np.concatenate([[True], ks[1:] != ks[:-1]]))
        for name, uf in (("min", np.minimum), ("max", np.maximum), ("xor", np.bitwise_xor)):
            ck, cv = O.collect_reduce(k, v, op=name)
            assert np.array_equal(ck, ks[starts])
            assert np.array_equal(cv, uf.reduceat(vs, starts)), name
        ck, cs = O.collect_reduce(k, v, op="sum")
        assert np.array_equal(cs, np.add.reduceat(vs, starts))  # uint64 adds wrap


def test_collect_reduce_first_and_last_in_input_order():
    # brute force: the value of each key's first / last record; and numpy's
    # np.unique first-occurrence index (on the array and on its reverse)
    rng = np.random.default_rng(53)
    for keys in _all_sequences(5):
        n = len(keys)
        vals = [int(x) for x in rng.integers(0, 2 ** 63, n, dtype=np.int64)]
        k = np.array(keys, dtype=np.uint64)
        v = np.array(vals, dtype=np.uint64)
        uniq = sorted(set(keys))
        fk, fv = O.collect_reduce(k, v, op="first")
        lk, lv = O.collect_reduce(k, v, op="last")
        assert [int(x) for x in fk] == uniq and [int(x) for x in lk] == uniq
        for j, u in enumerate(uniq):
            idx = [i for i in range(n) if keys[i] == u]
            assert int(fv[j]) == vals[idx[0]] and int(lv[j]) == vals[idx[-1]]
    for n, M in [(1, 1), (5000, 40), (50000, 20000)]:
        k = rng.integers(0, M, n, dtype=np.int64).astype(np.uint64)
        v = rng.integers(0, 2 ** 63, n, dtype=np.int64).astype(np.uint64)
        u, first = np.unique(k, return_index=True)
        _, rfirst = np.unique(k[::-1], return_index=True)
        fk, fv = O.collect_reduce(k, v, op="first")
        lk, lv = O.collect_reduce(k, v, op="last")
        assert np.array_equal(fk, u) and np.array_equal(fv, v[first])
        assert np.array_equal(lk, u) and np.array_equal(lv, v[::-1][rfirst])


def test_collect_reduce_affine_maps_compose_in_input_order():
    # each value is the map t -> a t + b mod 2^32 (a, b its high and low
    # halves); the result must act on any t as applying the key's maps one
    # after the other in input order
    rng = np.random.default_rng(61)
    M32 = 1 << 32
    for n, M in [(1, 1), (6, 2), (200, 5), (3000, 40)]:
        k = rng.integers(0, M, n, dtype=np.int64).astype(np.uint64)
        a = rng.integers(0, M32, n, dtype=np.uint64)
        b = rng.integers(0, M32, n, dtype=np.uint64)
        v = (a << np.uint64(32)) | b
        ck, cv = O.collect_reduce(k, v, op="affine")
        assert [int(x) for x in ck] == sorted(set(int(x) for x in k))
        for j, u in enumerate(ck):
            idx = [i for i in range(n) if k[i] == u]
            for t in (0, 1, 12345, M32 - 1):
                x = t
                for i in idx:
                    x = (int(a[i]) * x + int(b[i])) % M32
                r = int(cv[j])
                assert ((r >> 32) * t + (r & (M32 - 1))) % M32 == x
    # order matters: two maps of one key in either order give different folds
    k = np.array([3, 3], dtype=np.uint64)
    f, g = (2 << 32) | 1, (1 << 32) | 5
    assert int(O.collect_reduce(k, np.array([f, g], dtype=np.uint64), op="affine")[1][0]) != \
        int(O.collect_reduce(k, np.array([g, f], dtype=np.uint64), op="affine")[1][0])


def test_collect_reduce_monoid_identities():
    k = np.array([4, 9, 4, 9], dtype=np.uint64)
    v = np.array([MOD - 1, 0, MOD - 1, 0], dtype=np.uint64)
    # a value xor-ed with itself vanishes; min / max of equal values is that value
    assert [int(x) for x in O.collect_reduce(k, v, op="xor")[1]] == [0, 0]
    assert [int(x) for x in O.collect_reduce(k, v, op="min")[1]] == [MOD - 1, 0]
    assert [int(x) for x in O.collect_reduce(k, v, op="max")[1]] == [MOD - 1, 0]
    with pytest.raises(KeyError):
        O.collect_reduce(k, v, op="product")


def test_collect_reduce_wraps_mod_2_64():
    k = np.array([5, 5, 5], dtype=np.uint64)
    v = np.array([MOD - 1, MOD - 1, 3], dtype=np.uint64)
    ck, cs = O.collect_reduce(k, v)
    assert list(ck) == [5] and int(cs[0]) == (2 * (MOD - 1) + 3) % MOD


def test_random_medium_inputs_meet_the_definition():
    rng = np.random.default_rng(3)
    for n, M in [(1000, 10), (5000, 1000), (20000, 1 << 62)]:
        keys = rng.integers(0, M, n, dtype=np.int64).astype(np.uint64)
        v = np.arange(n, dtype=np.uint64)
        ko, vo = O.semisort_equal(keys, v)
        _check_semisort_equal([int(x) for x in keys], ko, vo)
        lo, lv = O.semisort_less(keys, v.astype(np.uint32))
        order = np.argsort(keys, kind="stable")
        assert np.array_equal(lv, order.astype(np.uint32)) and np.array_equal(lo, keys[order])
        hk, hc = O.histogram(keys)
        u, c = np.unique(keys, return_counts=True)
        assert np.array_equal(hk, u) and np.array_equal(hc, c.astype(np.uint64))


def test_identity_hash_orders_groups_by_key():
    keys = np.array([9, 3, 9, 1, 3, 3], dtype=np.uint64)
    ko, vo = O.semisort_equal(keys, np.arange(6, dtype=np.uint64), O.HASH_IDENTITY)
    assert list(ko) == [1, 3, 3, 3, 9, 9] and list(vo) == [3, 1, 4, 5, 0, 2]


# ----------------------------------------------------------- canonicalizer


def _groups_of(ko, vo):
    groups = []
    for p in range(len(ko)):
        if p == 0 or ko[p] != ko[p - 1]:
            groups.append([])
        groups[-1].append((int(ko[p]), int(vo[p])))
    return groups


def test_canonicalizer_accepts_every_group_order():
    keys = np.array([4, 2, 4, 7, 2, 9, 4, 11, 7], dtype=np.uint64)
    v = np.arange(keys.size, dtype=np.uint64)
    rk, rv = O.semisort_equal(keys, v)
    groups = _groups_of(rk, rv)
    assert len(groups) == 5
    for perm in itertools.permutations(groups):
        flat = [x for g in perm for x in g]
        ck_in = np.array([x[0] for x in flat], dtype=np.uint64)
        cv_in = np.array([x[1] for x in flat], dtype=np.uint64)
        bad, ck, cv = O.canonicalize_equal(ck_in, cv_in)
        assert bad == -1
        assert np.array_equal(ck, rk) and np.array_equal(cv, rv)


def test_canonicalizer_rejects_each_mutation():
    keys = np.array([4, 2, 4, 7, 2, 9, 4, 11, 7], dtype=np.uint64)
    v = np.arange(keys.size, dtype=np.uint64)
    rk, rv = O.semisort_equal(keys, v)
    flat = [(int(a), int(b)) for a, b in zip(rk, rv)]

    def canonical_ok(f):
        k = np.array([x[0] for x in f], dtype=np.uint64)
        w = np.array([x[1] for x in f], dtype=np.uint64)
        bad, ck, cv = O.canonicalize_equal(k, w)
        return bad == -1 and np.array_equal(ck, rk) and np.array_equal(cv, rv)

    assert canonical_ok(flat)
    # split a group: move the last record of the first multi-record group to the end
    p = next(i for i in range(1, len(flat)) if flat[i][0] == flat[i - 1][0])
    split = flat[:p] + flat[p + 1:] + [flat[p]]
    assert not canonical_ok(split)
    # swap two records inside a group (breaks stability)
    sw = list(flat)
    sw[p - 1], sw[p] = sw[p], sw[p - 1]
    assert not canonical_ok(sw)
    # duplicate one record over another
    dup = list(flat)
    dup[0] = dup[1] if dup[1][0] == dup[0][0] else dup[0]
    dup[-1] = dup[0]
    assert not canonical_ok(dup)
    # change a value
    cv = list(flat)
    cv[3] = (cv[3][0], cv[3][1] + 100)
    assert not canonical_ok(cv)


# ------------------------------------------------- Table 3 input statistics


def _stats_by_numpy(keys, thr):
    u, c = np.unique(keys, return_counts=True)
    return int(u.size), int(c.max()) if c.size else 0, int(c[c > thr].sum())


def test_stats_match_numpy_unique_counts_at_every_threshold():
    # Table 3 defines "Heavy Freq." as the share of records whose key occurs
    # MORE than 500 ln n times: a key whose count equals the threshold is
    # light.  Keys are built with known counts so that several of them sit
    # exactly at each threshold tried; a >= slip, a dropped run or a
    # miscounted last run changes the result.
    rng = np.random.default_rng(21)
    counts = {np.uint64(7): 5, np.uint64(1 << 63): 5, np.uint64(2): 4, np.uint64((1 << 64) - 1): 6,
              np.uint64(0): 1, np.uint64(99): 3, np.uint64(12345): 5}
    keys = np.concatenate([np.full(c, k, dtype=np.uint64) for k, c in counts.items()])
    keys = keys[rng.permutation(keys.size)]
    for thr in (0, 0.5, 1, 3, 4, 4.5, 5, 5.5, 6, 7):
        got = O.stats(keys, thr)
        assert got == _stats_by_numpy(keys, thr), thr
    # exactly at the threshold: the keys with count 5 are not heavy
    assert O.stats(keys, 5)[2] == 6
    assert O.stats(keys, 4.999)[2] == 5 * 3 + 6
    # the last run of the sorted keys (2^64 - 1) is counted
    assert O.stats(keys, 5)[1] == 6
    # empty and single-record inputs
    assert O.stats(np.zeros(0, dtype=np.uint64), 1) == (0, 0, 0)
    assert O.stats(np.array([5], dtype=np.uint64), 0) == (1, 1, 1)
    assert O.stats(np.array([5], dtype=np.uint64), 1) == (1, 1, 0)


def test_stats_on_random_skewed_keys_match_numpy():
    rng = np.random.default_rng(22)
    for trial in range(20):
        n = int(rng.integers(1, 5000))
        pool = rng.integers(0, 2 ** 63, int(rng.integers(1, 300)), dtype=np.int64).astype(np.uint64)
        pool[0] = np.uint64((1 << 64) - 1)
        keys = rng.choice(pool, n, p=rng.dirichlet(np.ones(pool.size) * 0.3))
        for thr in (0, 1, 10, 500 * math.log(max(n, 2)) / 100):
            assert O.stats(keys, thr) == _stats_by_numpy(keys, thr), (trial, thr)
        # thresholds equal to a count that occurs
        _, c = np.unique(keys, return_counts=True)
        for thr in np.unique(c)[:5]:
            assert O.stats(keys, float(thr)) == _stats_by_numpy(keys, float(thr)), (trial, thr)


# -------------------------------------------------- stage model of one level


def test_sample_indices_in_range_deterministic_and_uniform():
    idx = O.sample_indices(11, 0, 0, 1000, 20000)
    assert idx.max() < 1000
    assert np.array_equal(idx, O.sample_indices(11, 0, 0, 1000, 20000))
    assert not np.array_equal(idx[:100], O.sample_indices(11, 1, 0, 1000, 100))
    counts = np.bincount(idx.astype(np.int64), minlength=1000)
    chi2 = float(((counts - 20.0) ** 2 / 20.0).sum())
    assert chi2 < 999 + 6 * math.sqrt(2 * 999)


def test_sample_size_and_threshold_use_natural_log():
    # Section 3.6: |S| = 500 log n; natural log reproduces Table 3's heavy column
    assert O.sample_size(10 ** 9, 500) == math.ceil(500 * math.log(1e9))
    assert O.sample_size(5000, 500) == 5000 // 8  # capped for small subproblems
    assert O.heavy_threshold(10 ** 9) == 21
    assert O.heavy_threshold(16) == 3  # Fig. 2: 'more than 2 samples' with n = 16


def test_select_heavy_brute_force():
    rng = np.random.default_rng(5)
    s = rng.choice(np.array([3, 8, 8, 8, 1 << 40, 77, 77], dtype=np.uint64), 400)
    for tau in (1, 30, 60, 120):
        hk = O.select_heavy(s, tau)
        cnt = Counter(int(x) for x in s)
        want = sorted([k for k, c in cnt.items() if c >= tau], key=lambda k: (O.hash64(k), k))
        assert [int(x) for x in hk] == want


def test_select_heavy_bounded_table_keeps_the_most_frequent():
    # more keys reach tau than the table holds: tau rises to the least value
    # at which at most max_heavy keys reach it (checked by brute force over
    # every candidate threshold)
    rng = np.random.default_rng(8)
    for trial in range(30):
        pool = rng.integers(0, 2 ** 63, 40, dtype=np.int64).astype(np.uint64)
        s = rng.choice(pool, int(rng.integers(50, 600)), p=rng.dirichlet(np.ones(40) * 0.5))
        cnt = Counter(int(x) for x in s)
        for tau in (1, 2, 5):
            for cap in (1, 3, 7, 40):
                hk = [int(x) for x in O.select_heavy(s, tau, max_heavy=cap)]
                t = tau
                while sum(1 for c in cnt.values() if c >= t) > cap:
                    t += 1
                want = sorted([k for k, c in cnt.items() if c >= t], key=lambda k: (O.hash64(k), k))
                assert hk == want, (trial, tau, cap)
                assert len(hk) <= cap
                # nothing left out is more frequent than anything kept
                if hk:
                    assert min(cnt[k] for k in hk) > max([c for k, c in cnt.items() if k not in hk] or [0]) - 1


def test_count_prefix_distribute_against_definitions():
    rng = np.random.default_rng(9)
    n, tile = 10007, 1000
    keys = rng.integers(0, 3000, n, dtype=np.int64).astype(np.uint64)
    keys[rng.random(n) < 0.3] = 17  # one heavy key
    vals = np.arange(n, dtype=np.uint64)
    heavy = O.select_heavy(keys[rng.integers(0, n, 500)], 40)
    assert 17 in [int(x) for x in heavy]
    nl_bits = 4
    nb = (1 << nl_bits) + heavy.size
    bids = O.bucket_ids(keys, heavy, nl_bits, 0)
    # bucket ids: heavy keys get n_L + rank, light keys the low hash bits
    for j in range(0, n, 97):
        k = int(keys[j])
        if k in [int(x) for x in heavy]:
            assert bids[j] == (1 << nl_bits) + [int(x) for x in heavy].index(k)
        else:
            assert bids[j] == O.hash64(k) & ((1 << nl_bits) - 1)
    C = O.count_matrix(bids, tile, nb)
    tiles = (n + tile - 1) // tile
    for i in range(tiles):
        seg = bids[i * tile:(i + 1) * tile].astype(np.int64)
        assert np.array_equal(C[i], np.bincount(seg, minlength=nb).astype(np.uint32))
    X, off = O.column_prefix(C, n)
    flat = C.T.reshape(-1).astype(np.int64)  # column-major walk
    excl = np.concatenate([[0], np.cumsum(flat)[:-1]])
    assert np.array_equal(X.T.reshape(-1), excl.astype(np.uint32))
    assert off[-1] == n and np.all(np.diff(off.astype(np.int64)) >= 0)
    tk, tv = O.distribute(keys, vals, bids, tile, nb, X)
    order = np.argsort(bids, kind="stable")  # a stable counting sort by bucket id
    assert np.array_equal(tv, order.astype(np.uint64)) and np.array_equal(tk, keys[order])
    # each heavy bucket holds exactly one key
    for h in range(heavy.size):
        a, b = int(off[(1 << nl_bits) + h]), int(off[(1 << nl_bits) + h + 1])
        assert np.all(tk[a:b] == heavy[h])


def _random_csr(rng, nv, ne, sort_rows=False, unique=False):
    if unique:
        pairs = rng.choice(nv * nv, size=min(ne, nv * nv), replace=False)
        src, dst = pairs // nv, pairs % nv
    else:
        src = rng.integers(0, nv, ne)
        dst = rng.integers(0, nv, ne)
    o = np.lexsort((dst, src)) if sort_rows else np.argsort(src, kind="stable")
    src, dst = src[o], dst[o]
    offs = np.zeros(nv + 1, dtype=np.uint64)
    np.add.at(offs, src + 1, 1)
    return np.cumsum(offs).astype(np.uint64), dst.astype(np.uint32)


def test_transpose_csr_brute_force():
    # E^T lists, for every vertex v, the first endpoints u of the edges (u, v)
    # in input order
    rng = np.random.default_rng(41)
    for nv, ne in [(1, 0), (1, 3), (2, 5), (5, 0), (5, 12), (7, 40), (30, 200)]:
        offs, cols = _random_csr(rng, nv, ne)
        oo, oc = O.transpose_csr(offs, cols)
        lists = [[] for _ in range(nv)]
        for u in range(nv):
            for e in range(int(offs[u]), int(offs[u + 1])):
                lists[int(cols[e])].append(u)
        assert [int(x) for x in oo] == [0] + list(np.cumsum([len(x) for x in lists]))
        assert [int(x) for x in oc] == [u for x in lists for u in x]


def test_transpose_csr_matches_scipy_and_is_an_involution():
    sp = pytest.importorskip("scipy.sparse")
    rng = np.random.default_rng(43)
    for nv, ne in [(50, 300), (1000, 20000), (3000, 3000)]:
        offs, cols = _random_csr(rng, nv, ne, sort_rows=True, unique=True)
        oo, oc = O.transpose_csr(offs, cols)
        a = sp.csr_matrix((np.ones(cols.size), cols.astype(np.int64), offs.astype(np.int64)), shape=(nv, nv))
        t = a.T.tocsr()
        t.sort_indices()
        assert np.array_equal(oo, t.indptr.astype(np.uint64))
        assert np.array_equal(oc, t.indices.astype(np.uint32))
        bo, bc = O.transpose_csr(oo, oc)
        assert np.array_equal(bo, offs) and np.array_equal(bc, cols)


def test_transpose_csr_rejects_an_invalid_graph():
    with pytest.raises(ValueError):
        O.transpose_csr(np.array([0, 2], dtype=np.uint64), np.array([0, 1], dtype=np.uint32))  # target >= nv
    with pytest.raises(ValueError):
        O.transpose_csr(np.array([0, 3, 2], dtype=np.uint64), np.array([0, 1], dtype=np.uint32))


def test_oracle_on_32bit_extremes_exhaustive():
    # 32-bit keys are zero-extended for the oracle: every sequence of length
    # <= 6 over the uint32 extremes gives a stable grouping (semisort_=) and a
    # stable sort (semisort_<, against numpy's stable argsort)
    import itertools
    ext = [0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF]
    for n in range(0, 7):
        for seq in itertools.product(ext, repeat=n) if n <= 4 else [tuple(np.random.default_rng(n).choice(ext, n))]:
            k = np.array(seq, dtype=np.uint32).astype(np.uint64)
            v = np.arange(n, dtype=np.uint64)
            ok, ov = O.semisort_equal(k, v)
            assert sorted(ov.tolist()) == list(range(n))
            assert np.array_equal(k[ov], ok)
            seen = set()
            for i in range(n):
                if i == 0 or ok[i] != ok[i - 1]:
                    assert int(ok[i]) not in seen
                    seen.add(int(ok[i]))
                else:
                    assert ov[i] > ov[i - 1]
            lk, lv = O.semisort_less(k, v)
            o = np.argsort(k, kind="stable")
            assert np.array_equal(lk, k[o]) and np.array_equal(lv, v[o])


# ---- 128-bit keys (Section 2.1: any key type with an equality test) ----------

def _is_stable_grouping_wide(keys, vals, ok, ov):
    """Brute-force definition for index values: a permutation of the input in
    which every record kept its key, equal keys are contiguous, and records of
    a key keep their input order."""
    n = keys.shape[0]
    if sorted(ov.tolist()) != list(range(n)):
        return False
    if not np.array_equal(keys[ov.astype(np.int64)], ok):
        return False
    seen = set()
    for i in range(n):
        k = (int(ok[i, 0]), int(ok[i, 1]))
        if i == 0 or k != (int(ok[i - 1, 0]), int(ok[i - 1, 1])):
            if k in seen:
                return False
            seen.add(k)
        elif ov[i] <= ov[i - 1]:
            return False
    return True


def test_wide_oracle_exhaustive_tiny():
    # every sequence of up to 7 keys over four 128-bit keys that pairwise agree
    # in one word (equal low or equal high word), so comparing one word only
    # merges two keys and fails; the output is the unique stable grouping in
    # ascending key order
    alphabet = [(1, 0), (0, 1), (1, 1), (0, 0)]
    for n in range(0, 8):
        for seq in itertools.product(range(4), repeat=n):
            k = np.array([alphabet[x] for x in seq], dtype=np.uint64).reshape(n, 2)
            v = np.arange(n, dtype=np.uint64)
            ok, ov = O.semisort_equal_wide(k, v)
            assert _is_stable_grouping_wide(k, v, ok, ov), seq
            as_int = [int(a) + (int(b) << 64) for a, b in ok.tolist()]
            assert as_int == sorted(as_int), seq
            bad, ck, cv = O.canonicalize_equal_wide(ok, ov)
            assert bad == -1 and np.array_equal(ck, ok) and np.array_equal(cv, ov)


def test_wide_oracle_reduces_to_a_stable_sort_of_either_word():
    # with one word constant the result is a stable sort by the other word
    # (numpy's stable argsort); u32 values move with their records
    rng = np.random.default_rng(41)
    n = 20_000
    w = rng.integers(0, 300, n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    v = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    for lo_varies in (True, False):
        k = np.zeros((n, 2), dtype=np.uint64)
        k[:, 0 if lo_varies else 1] = w
        k[:, 1 if lo_varies else 0] = 12345
        ok, ov = O.semisort_equal_wide(k, v)
        o = np.argsort(w, kind="stable")
        assert np.array_equal(ok, k[o]) and np.array_equal(ov, v[o])


def test_wide_oracle_groups_match_python_grouping():
    # random keys drawn from few high and low words: the groups (as lists of
    # input indices) equal those a Python dict builds in one pass
    rng = np.random.default_rng(42)
    n = 5_000
    k = np.stack([rng.integers(0, 7, n, dtype=np.uint64), rng.integers(0, 5, n, dtype=np.uint64)], axis=1)
    v = np.arange(n, dtype=np.uint64)
    ok, ov = O.semisort_equal_wide(k, v)
    groups = {}
    for i, (a, b) in enumerate(k.tolist()):
        groups.setdefault((b, a), []).append(i)
    want = [i for key in sorted(groups) for i in groups[key]]
    assert ov.tolist() == want


def test_wide_canonicalizer_detects_split_runs_and_restores_order():
    a, b, c = (5, 9), (5, 10), (6, 9)  # a and b differ in the high word only, a and c in the low word only
    for seq, bad_at in (([a, b, a], 2), ([a, c, a], 2), ([b, b, a, c, b], 4), ([a, a, b, c], -1)):
        k = np.array(seq, dtype=np.uint64)
        v = np.arange(len(seq), dtype=np.uint64)
        bad, _, _ = O.canonicalize_equal_wide(k, v)
        assert bad == bad_at, seq
    # any order of the groups of a valid result canonicalizes to the oracle's
    rng = np.random.default_rng(43)
    n = 3000
    k = np.stack([rng.integers(0, 4, n, dtype=np.uint64), rng.integers(0, 4, n, dtype=np.uint64)], axis=1)
    v = np.arange(n, dtype=np.uint64)
    ok, ov = O.semisort_equal_wide(k, v)
    starts = [0] + [i for i in range(1, n) if tuple(ok[i]) != tuple(ok[i - 1])] + [n]
    runs = [list(range(starts[j], starts[j + 1])) for j in range(len(starts) - 1)]
    rng.shuffle(runs)
    perm = np.array([i for r in runs for i in r])
    bad, ck, cv = O.canonicalize_equal_wide(ok[perm], ov[perm])
    assert bad == -1 and np.array_equal(ck, ok) and np.array_equal(cv, ov)


# ---- the 2 x 2 matrix product monoid (a non-commutative fold, Section 3.5) ----

def _mat(a, b, c, d):
    return np.uint64(a | (b << 16) | (c << 32) | (d << 48))


def test_mat2_monoid_special_cases_and_order():
    rng = np.random.default_rng(61)
    n = 6000
    keys = rng.integers(0, 40, n, dtype=np.uint64)
    # diagonal matrices: the fold is the product of each diagonal entry mod 2^16
    a = rng.integers(0, 1 << 16, n)
    d = rng.integers(0, 1 << 16, n)
    vals = np.array([_mat(int(x), 0, 0, int(y)) for x, y in zip(a, d)], dtype=np.uint64)
    ok, ov = O.collect_reduce(keys, vals, op="mat2")
    for k, v in zip(ok.tolist(), ov.tolist()):
        sel = np.nonzero(keys == k)[0]
        pa = pd = 1
        for i in sel:
            pa = pa * int(a[i]) % 65536
            pd = pd * int(d[i]) % 65536
        assert v == int(_mat(pa, 0, 0, pd)), k
    # unipotent upper-triangular matrices (1, x; 0, 1): the fold adds the x
    x = rng.integers(0, 1 << 16, n)
    vals = np.array([_mat(1, int(t), 0, 1) for t in x], dtype=np.uint64)
    ok, ov = O.collect_reduce(keys, vals, op="mat2")
    for k, v in zip(ok.tolist(), ov.tolist()):
        s = int(x[keys == k].sum()) % 65536
        assert v == int(_mat(1, s, 0, 1)), k
    # order: (1,1;0,1)(1,0;1,1) = (2,1;1,1), the other order gives (1,1;1,2)
    A, B = _mat(1, 1, 0, 1), _mat(1, 0, 1, 1)
    ok, ov = O.collect_reduce(np.array([5, 5, 9], dtype=np.uint64), np.array([A, B, B], dtype=np.uint64), op="mat2")
    assert ok.tolist() == [5, 9]
    assert ov.tolist() == [int(_mat(2, 1, 1, 1)), int(B)]
    ok, ov = O.collect_reduce(np.array([5, 5], dtype=np.uint64), np.array([B, A], dtype=np.uint64), op="mat2")
    assert ov.tolist() == [int(_mat(1, 1, 1, 2))]
