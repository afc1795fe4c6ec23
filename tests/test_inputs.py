"""Pins for the seeded input generators: the distributions' parameterization is
checked against the statistics Table 3 prints (closed-form expectations at
n = 10^9) and the draws against their probability mass functions."""
import json
import math
import os

import numpy as np
import pytest

from paper_2304_10078_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))


def _zipf_norm(s, N, K=10 ** 6):
    # sum_{k<=N} k^-s: exact head plus a midpoint integral for the tail
    head = float(np.sum(np.arange(1, K + 1, dtype=np.float64) ** -s))
    a, b = K + 0.5, N + 0.5
    tail = (b ** (1 - s) - a ** (1 - s)) / (1 - s) if s != 1 else math.log(b / a)
    return head + tail


def _zipf_expected(s, N, n):
    Z = _zipf_norm(s, N)
    T = 500 * math.log(n)
    # keys k with n * k^-s / Z > T are the heavy ones: k < (n / (Z T))^(1/s)
    kstar = int(math.floor((n / (Z * T)) ** (1.0 / s)))
    while kstar > 0 and n * kstar ** -s / Z <= T:
        kstar -= 1
    heavy = float(np.sum(np.arange(1, kstar + 1, dtype=np.float64) ** -s)) / Z if kstar else 0.0
    return n / Z, heavy


def _exp_expected(lam, n):
    p0 = 1 - math.exp(-lam)
    T = 500 * math.log(n)
    # P(key = k) = e^{-lam k} p0; heavy keys are those with n P(k) > T
    if n * p0 <= T:
        return n * p0, 0.0
    kstar = math.floor(math.log(n * p0 / T) / lam)
    return n * p0, 1 - math.exp(-lam * (kstar + 1))


def test_distribution_parameters_reproduce_table3_columns():
    g = json.load(open(os.path.join(HERE, "golden", "table3_input_stats.json")))
    n = g["n"]
    for row in g["rows"]:
        if row["dist"] == "zipf":
            mx, hv = _zipf_expected(row["param"], 10 ** 9, n)
        else:
            mx, hv = _exp_expected(row["param"], n)
        assert abs(mx - row["max_freq"]) <= 0.01 * row["max_freq"], row
        assert abs(hv - row["heavy_frac"]) <= 0.0015 + 0.01 * row["heavy_frac"], row


def test_zipf_draws_follow_the_pmf():
    n, s, N = 400000, 1.2, 10 ** 9
    z = I.np_zipf(n, s, N, seed=4)
    assert z.min() >= 1 and z.max() <= N
    Z = _zipf_norm(s, N)
    for k in range(1, 9):
        p = k ** -s / Z
        got = float(np.sum(z == k))
        assert abs(got - n * p) < 5 * math.sqrt(n * p * (1 - p)), k


def test_exponential_and_uniform_draws():
    n = 400000
    e = I.np_exponential(n, 1e-3, seed=5)
    p0 = 1 - math.exp(-1e-3)
    assert abs(float(np.sum(e == 0)) - n * p0) < 5 * math.sqrt(n * p0)
    assert abs(float(e.mean()) - (math.exp(-1e-3) / p0)) < 0.02 * (1 / 1e-3)
    u = I.np_uniform(n, 1000, seed=3)
    assert u.max() < 1000
    c = np.bincount(u.astype(np.int64), minlength=1000)
    chi2 = float(((c - n / 1000) ** 2 / (n / 1000)).sum())
    assert chi2 < 999 + 6 * math.sqrt(2 * 999)


def test_numpy_and_torch_back_ends_draw_the_same_integers():
    torch = pytest.importorskip("torch")
    idx = torch.arange(0, 5000, dtype=torch.int64)
    a = I.np_u64(9, 2, np.arange(5000, dtype=np.uint64))
    b = I.t_u64(9, 2, idx).numpy().view(np.uint64)
    assert np.array_equal(a, b)
    assert np.array_equal(I.np_uniform(5000, 10 ** 9, 2), I.t_uniform(5000, 10 ** 9, 2, "cpu").numpy().view(np.uint64))
    assert np.array_equal(I.np_rehash(a), I.t_rehash(torch.from_numpy(a.view(np.int64))).numpy().view(np.uint64))


def test_workloads_are_seeded_and_shaped():
    k, v = I.np_workload("uniform1e5_index", 10000, 1)
    assert k.dtype == np.uint64 and v.dtype == np.uint64 and np.array_equal(v, np.arange(10000))
    k2, _ = I.np_workload("uniform1e5_index", 10000, 1)
    assert np.array_equal(k, k2)
    k3, v3 = I.np_workload("exp1e-5_u32idx", 1000, 5)
    assert v3.dtype == np.uint32


def test_batch_sizes_follow_the_batched_configuration():
    # 4096 log-uniform sizes in [1e3, 1e7], scaled to a total of at most 5e8,
    # clamped at 1e3
    sz = I.batch_sizes(4096, 1e3, 1e7, 5e8, 7)
    assert sz.sum() <= 5e8 and sz.sum() > 0.99 * 5e8
    assert sz.min() == 1000 and sz.max() < 1e7 * 0.2
    # log-uniform before scaling: log10 of the unclamped sizes spreads evenly
    u = np.log10(sz[sz > 1000])
    assert np.ptp(u) > 2.5
    d = I.batch_dists(4096, 7)
    cnt = np.bincount(d, minlength=4)
    assert cnt.sum() == 4096 and cnt.min() > 900


def test_batch_workload_numpy_and_torch_agree():
    torch = pytest.importorskip("torch")
    k, v, o, d = I.np_batch_workload(24, 1e3, 2e4, 1e5, 3)
    tk, tv, to, td = I.t_batch_workload(24, 1e3, 2e4, 1e5, 3, "cpu")
    assert np.array_equal(o, to) and np.array_equal(d, td)
    assert np.array_equal(tk.numpy().view(np.uint64), k)
    assert np.array_equal(tv.numpy().view(np.uint64), v)
    # each instance draws from its own distribution: uniform[0, n/10) keys stay below n/10
    for i in range(24):
        a, b = int(o[i]), int(o[i + 1])
        if d[i] == 0:
            assert k[a:b].max() < max(1, (b - a) // 10)
        if d[i] == 3:
            assert k[a:b].max() < 100


def test_graph_generators_are_valid_csr_and_agree_across_back_ends():
    torch = pytest.importorskip("torch")
    for kind in I.GRAPH_KINDS:
        for nv, ne in [(1, 5), (97, 1000), (1000, 30000)]:
            offs, cols = I.np_graph(kind, nv, ne, 11)
            assert offs.size == nv + 1 and int(offs[0]) == 0 and int(offs[-1]) == ne
            assert np.all(np.diff(offs.astype(np.int64)) >= 0)
            assert cols.size == ne and (ne == 0 or int(cols.max()) < nv)
            to, tc = I.t_graph(kind, nv, ne, 11, "cpu")
            assert np.array_equal(offs.view(np.int64), to.numpy()) and np.array_equal(cols.view(np.int32), tc.numpy())
    offs, cols = I.np_graph("knn", 1000, 30000, 11)
    rows = np.repeat(np.arange(1000), np.diff(offs.astype(np.int64)))
    d = (cols.astype(np.int64) - rows) % 1000
    assert np.all((d <= I.KNN_WIDTH) | (d >= 1000 - I.KNN_WIDTH))


def test_32bit_key_workloads():
    # uint32 keys; the 32-bit mixer is a bijection (no two ranks collide), and
    # the numpy and torch back ends give the same bits
    import torch
    for name in ("zipf1.2_hashed_k32", "uniform1e9_k32", "exp1e-5_k32_u32idx"):
        k, v = I.np_workload(name, 100_000, 3)
        assert k.dtype == np.uint32 and I.key_bytes(name) == 4
        tk, tv = I.t_workload(name, 100_000, 3, "cpu")
        assert np.array_equal(k, tk.numpy().view(np.uint32))
    x = np.arange(1 << 20, dtype=np.uint32) * np.uint32(2654435761)
    assert np.unique(I.np_fmix32(x)).size == x.size
    z = I.np_zipf(200_000, 1.2, 10 ** 9, 3, 0)
    assert np.unique(I.np_fmix32(z.astype(np.uint32))).size == np.unique(z).size


def test_128bit_key_workloads():
    # (n, 2) words; the numpy and torch back ends give the same bits; the low
    # word is the distribution's key, so distinct keys stay distinct
    for name in ("zipf1.2_hashed_k128", "uniform1e9_k128"):
        k, v = I.np_workload(name, 50_000, 5)
        assert k.shape == (50_000, 2) and k.dtype == np.uint64 and I.key_bytes(name) == 16
        tk, tv = I.t_workload(name, 50_000, 5, "cpu")
        assert np.array_equal(k, tk.numpy().view(np.uint64)) and np.array_equal(v, tv.numpy().view(v.dtype))
        assert np.unique(k[:, 0]).size == np.unique(k, axis=0).shape[0]
