/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain single-threaded CPU reference for semisort, histogram and
 * collect-reduce (Dong et al., SPAA 2023).  The definitional functions follow
 * Section 2.1 (problem definitions) and Section 2.2 (stability) and reach their
 * result with a library sort; the stage functions follow the steps of
 * Algorithm 1 (Sections 3.1 and 3.2) in the paper's order and notation.
 * Nothing here is blocked, fused or reordered.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- hashing ---------------------------------------------------------- */

/* The 64-bit finalizer ("fmix64") that Austin Appleby published with
 * MurmurHash3: xor-shift by 33, multiply by an odd constant, twice, then a
 * last xor-shift.  Every step is invertible, so the map is a bijection and
 * equal hashes mean equal keys. */
static uint64_t murmur3_fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

uint64_t orc_hash(uint64_t k, int hash_mode)
{
    return hash_mode == 1 ? k : murmur3_fmix64(k);
}

/* SplitMix64's output function (Steele, Lea, Flood 2014). */
uint64_t orc_splitmix_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* ---- small helpers ----------------------------------------------------- */

static uint64_t load_val(const void* vals, uint32_t vb, uint64_t i)
{
    if (vb == 4) return ((const uint32_t*)vals)[i];
    return ((const uint64_t*)vals)[i];
}

static void store_val(void* vals, uint32_t vb, uint64_t i, uint64_t v)
{
    if (vb == 4) ((uint32_t*)vals)[i] = (uint32_t)v;
    else ((uint64_t*)vals)[i] = v;
}

typedef struct { uint64_t h, k, i; } hki_t;

static int cmp_hki(const void* a, const void* b)
{
    const hki_t* x = (const hki_t*)a;
    const hki_t* y = (const hki_t*)b;
    if (x->h != y->h) return x->h < y->h ? -1 : 1;
    if (x->k != y->k) return x->k < y->k ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    return 0;
}

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* ---- plain definitions (Section 2.1, stability from Section 2.2) ------- */

int orc_semisort_equal(const uint64_t* keys, const void* vals, uint32_t vb, uint64_t n,
                       int hash_mode, uint64_t* keys_out, void* vals_out)
{
    /* Sorting by (h(k), k, i) puts equal keys together (contiguity), keeps
     * their input order (the index breaks ties: stability) and fixes one
     * group order, ascending (h(k), k), so the result is unique. */
    if (n == 0) return 0;
    hki_t* t = (hki_t*)malloc(n * sizeof(hki_t));
    if (!t) return -1;
    for (uint64_t i = 0; i < n; i++) {
        t[i].h = orc_hash(keys[i], hash_mode);
        t[i].k = keys[i];
        t[i].i = i;
    }
    qsort(t, n, sizeof(hki_t), cmp_hki);
    for (uint64_t p = 0; p < n; p++) {
        keys_out[p] = keys[t[p].i];
        store_val(vals_out, vb, p, load_val(vals, vb, t[p].i));
    }
    free(t);
    return 0;
}

int orc_semisort_less(const uint64_t* keys, const void* vals, uint32_t vb, uint64_t n,
                      uint64_t* keys_out, void* vals_out)
{
    /* Ascending groups plus stability: a stable sort by key, done as a sort
     * by (k, i). */
    if (n == 0) return 0;
    hki_t* t = (hki_t*)malloc(n * sizeof(hki_t));
    if (!t) return -1;
    for (uint64_t i = 0; i < n; i++) {
        t[i].h = keys[i];
        t[i].k = keys[i];
        t[i].i = i;
    }
    qsort(t, n, sizeof(hki_t), cmp_hki);
    for (uint64_t p = 0; p < n; p++) {
        keys_out[p] = keys[t[p].i];
        store_val(vals_out, vb, p, load_val(vals, vb, t[p].i));
    }
    free(t);
    return 0;
}

int64_t orc_histogram(const uint64_t* keys, uint64_t n, uint64_t* out_keys,
                      uint64_t* out_counts)
{
    /* G = { (k, |{r : key(r) = k}|) } over the unique keys k. */
    if (n == 0) return 0;
    uint64_t* s = (uint64_t*)malloc(n * sizeof(uint64_t));
    if (!s) return -1;
    memcpy(s, keys, n * sizeof(uint64_t));
    qsort(s, n, sizeof(uint64_t), cmp_u64);
    int64_t m = 0;
    uint64_t p = 0;
    while (p < n) {
        uint64_t q = p;
        while (q < n && s[q] == s[p]) q++;
        out_keys[m] = s[p];
        out_counts[m] = q - p;
        m++;
        p = q;
    }
    free(s);
    return m;
}

typedef struct { uint64_t k, v; } kv_t;

static int cmp_kv_key(const void* a, const void* b)
{
    const kv_t* x = (const kv_t*)a;
    const kv_t* y = (const kv_t*)b;
    return x->k < y->k ? -1 : (x->k > y->k ? 1 : 0);
}

int64_t orc_collect_reduce(const uint64_t* keys, const uint64_t* vals, uint64_t n,
                           uint64_t* out_keys, uint64_t* out_sums)
{
    /* R = { (k, sum over r in S_k of M(r)) } with M(r) = value(r) and the
     * monoid (+ mod 2^64, 0).  Addition mod 2^64 is associative and
     * commutative, so the summation order does not change the result. */
    if (n == 0) return 0;
    kv_t* s = (kv_t*)malloc(n * sizeof(kv_t));
    if (!s) return -1;
    for (uint64_t i = 0; i < n; i++) {
        s[i].k = keys[i];
        s[i].v = vals[i];
    }
    qsort(s, n, sizeof(kv_t), cmp_kv_key);
    int64_t m = 0;
    uint64_t p = 0;
    while (p < n) {
        uint64_t acc = 0; /* identity I = 0 */
        uint64_t q = p;
        while (q < n && s[q].k == s[p].k) {
            acc += s[q].v; /* unsigned: wraps mod 2^64 */
            q++;
        }
        out_keys[m] = s[p].k;
        out_sums[m] = acc;
        m++;
        p = q;
    }
    free(s);
    return m;
}

/* The monoids of collect-reduce on uint64 values (Section 3.5 allows any
 * monoid (+, I)): 0 = (+ mod 2^64, 0), 1 = (min, 2^64 - 1), 2 = (max, 0),
 * 3 = (xor, 0).  All four are associative and commutative. */
static uint64_t monoid_identity(int op)
{
    return op == 1 ? ~0ULL : 0ULL;
}

static uint64_t monoid_combine(int op, uint64_t x, uint64_t y)
{
    switch (op) {
    case 0: return x + y;
    case 1: return x < y ? x : y;
    case 2: return x > y ? x : y;
    default: return x ^ y;
    }
}

typedef struct { uint64_t k, i; } ki_t;

static int cmp_ki(const void* a, const void* b)
{
    const ki_t* x = (const ki_t*)a;
    const ki_t* y = (const ki_t*)b;
    if (x->k != y->k) return x->k < y->k ? -1 : 1;
    return x->i < y->i ? -1 : (x->i > y->i ? 1 : 0);
}

/* 6: composition of affine maps on 32-bit integers.  A value holds (a, b) =
 * (high, low 32 bits) for t -> a t + b mod 2^32; x (+) y applies x, then y:
 * (a_y a_x, a_y b_x + b_y) mod 2^32, identity (1, 0). */
static uint64_t affine_then(uint64_t x, uint64_t y)
{
    const uint32_t ax = (uint32_t)(x >> 32), bx = (uint32_t)x;
    const uint32_t ay = (uint32_t)(y >> 32), by = (uint32_t)y;
    const uint32_t a = ay * ax, b = ay * bx + by;
    return ((uint64_t)a << 32) | b;
}

/* 7: products of 2 x 2 matrices over the integers mod 2^16.  A value holds
 * the entries (a, b; c, d) as its 16-bit fields from the low end; x (+) y is
 * the matrix product x y, identity (1, 0; 0, 1).  Associative (matrix
 * multiplication is), not commutative. */
static uint64_t mat2_mul(uint64_t x, uint64_t y)
{
    const uint32_t xa = (uint16_t)x, xb = (uint16_t)(x >> 16), xc = (uint16_t)(x >> 32), xd = (uint16_t)(x >> 48);
    const uint32_t ya = (uint16_t)y, yb = (uint16_t)(y >> 16), yc = (uint16_t)(y >> 32), yd = (uint16_t)(y >> 48);
    const uint64_t a = (uint16_t)(xa * ya + xb * yc), b = (uint16_t)(xa * yb + xb * yd);
    const uint64_t c = (uint16_t)(xc * ya + xd * yc), d = (uint16_t)(xc * yb + xd * yd);
    return a | (b << 16) | (c << 32) | (d << 48);
}

/* Non-commutative monoids (Section 3.5: a stable algorithm folds any
 * associative operation): 4 = first (x (+) y = x), 5 = last (x (+) y = y),
 * 6 = affine composition, 7 = 2 x 2 matrix product, folded over each key's
 * records in input order. */
static int64_t collect_reduce_in_order(const uint64_t* keys, const uint64_t* vals, uint64_t n, int op,
                                       uint64_t* out_keys, uint64_t* out_vals)
{
    ki_t* s = (ki_t*)malloc(n * sizeof(ki_t));
    if (!s) return -1;
    for (uint64_t i = 0; i < n; i++) {
        s[i].k = keys[i];
        s[i].i = i;
    }
    qsort(s, n, sizeof(ki_t), cmp_ki); /* by (key, input position): each key's records in input order */
    int64_t m = 0;
    uint64_t p = 0;
    while (p < n) {
        uint64_t acc = vals[s[p].i];
        uint64_t q = p + 1;
        while (q < n && s[q].k == s[p].k) {
            acc = op == 4 ? acc : op == 5 ? vals[s[q].i] : op == 6 ? affine_then(acc, vals[s[q].i])
                                                                   : mat2_mul(acc, vals[s[q].i]);
            q++;
        }
        out_keys[m] = s[p].k;
        out_vals[m] = acc;
        m++;
        p = q;
    }
    free(s);
    return m;
}

int64_t orc_collect_reduce_monoid(const uint64_t* keys, const uint64_t* vals, uint64_t n, int op,
                                  uint64_t* out_keys, uint64_t* out_vals)
{
    /* R = { (k, fold of the monoid over M(r), r in S_k) } with M(r) =
     * value(r); ascending keys. */
    if (op < 0 || op > 7) return -2;
    if (op >= 4) return n ? collect_reduce_in_order(keys, vals, n, op, out_keys, out_vals) : 0;
    if (n == 0) return 0;
    kv_t* s = (kv_t*)malloc(n * sizeof(kv_t));
    if (!s) return -1;
    for (uint64_t i = 0; i < n; i++) {
        s[i].k = keys[i];
        s[i].v = vals[i];
    }
    qsort(s, n, sizeof(kv_t), cmp_kv_key);
    int64_t m = 0;
    uint64_t p = 0;
    while (p < n) {
        uint64_t acc = monoid_identity(op);
        uint64_t q = p;
        while (q < n && s[q].k == s[p].k) {
            acc = monoid_combine(op, acc, s[q].v);
            q++;
        }
        out_keys[m] = s[p].k;
        out_vals[m] = acc;
        m++;
        p = q;
    }
    free(s);
    return m;
}

int orc_transpose_csr(uint64_t nv, uint64_t ne, const uint64_t* offs, const uint32_t* cols,
                      uint64_t* out_offs, uint32_t* out_cols)
{
    /* E^T = { (u, v) : (v, u) in E } (Section 5, graph transposing), in CSR:
     * out_offs[v] = number of edges whose other endpoint is below v, and the
     * edges into v listed in input order (first endpoints ascending for a
     * row-ordered input), i.e. a stable counting sort of the edges by their
     * other endpoint. */
    if (offs[0] != 0 || offs[nv] != ne) return -2;
    for (uint64_t u = 0; u < nv; u++)
        if (offs[u + 1] < offs[u]) return -2;
    for (uint64_t e = 0; e < ne; e++)
        if (cols[e] >= nv) return -2;
    uint64_t* next = (uint64_t*)calloc(nv + 1, sizeof(uint64_t));
    if (!next) return -1;
    for (uint64_t e = 0; e < ne; e++) next[cols[e] + 1]++;
    for (uint64_t v = 0; v < nv; v++) next[v + 1] += next[v];
    memcpy(out_offs, next, (nv + 1) * sizeof(uint64_t));
    for (uint64_t u = 0; u < nv; u++)
        for (uint64_t e = offs[u]; e < offs[u + 1]; e++) out_cols[next[cols[e]]++] = (uint32_t)u;
    free(next);
    return 0;
}

typedef struct { uint64_t h, k, start, len; } run_t;

static int cmp_run(const void* a, const void* b)
{
    const run_t* x = (const run_t*)a;
    const run_t* y = (const run_t*)b;
    if (x->h != y->h) return x->h < y->h ? -1 : 1;
    if (x->k != y->k) return x->k < y->k ? -1 : 1;
    if (x->start != y->start) return x->start < y->start ? -1 : 1;
    return 0;
}

int64_t orc_canonicalize_equal(const uint64_t* keys, const void* vals, uint32_t vb,
                               uint64_t n, int hash_mode, uint64_t* canon_keys,
                               void* canon_vals)
{
    if (n == 0) return -1;
    uint64_t nruns = 1;
    for (uint64_t p = 1; p < n; p++)
        if (keys[p] != keys[p - 1]) nruns++;
    run_t* r = (run_t*)malloc(nruns * sizeof(run_t));
    if (!r) return -2;
    uint64_t j = 0, p = 0;
    while (p < n) {
        uint64_t q = p;
        while (q < n && keys[q] == keys[p]) q++;
        r[j].h = orc_hash(keys[p], hash_mode);
        r[j].k = keys[p];
        r[j].start = p;
        r[j].len = q - p;
        j++;
        p = q;
    }
    qsort(r, nruns, sizeof(run_t), cmp_run);
    /* Two runs with one key sit next to each other after the sort; the later
     * one is where contiguity broke. */
    int64_t bad = -1;
    for (uint64_t x = 1; x < nruns; x++) {
        if (r[x].k == r[x - 1].k) {
            if (bad < 0 || (int64_t)r[x].start < bad) bad = (int64_t)r[x].start;
        }
    }
    if (bad >= 0) {
        free(r);
        return bad;
    }
    uint64_t o = 0;
    for (uint64_t x = 0; x < nruns; x++) {
        for (uint64_t y = 0; y < r[x].len; y++) {
            canon_keys[o] = keys[r[x].start + y];
            store_val(canon_vals, vb, o, load_val(vals, vb, r[x].start + y));
            o++;
        }
    }
    free(r);
    return -1;
}

/* ---- 128-bit keys ------------------------------------------------------ */
/* Section 2.1 takes keys of any type with an equality test.  A 128-bit key j
 * is the pair (keys[2j], keys[2j + 1]) = (low word, high word); two keys are
 * equal when both words are. */

typedef struct { uint64_t hi, lo, i; } wki_t;

static int cmp_wki(const void* a, const void* b)
{
    const wki_t* x = (const wki_t*)a;
    const wki_t* y = (const wki_t*)b;
    if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
    if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    return 0;
}

int orc_semisort_equal_wide(const uint64_t* keys, const void* vals, uint32_t vb, uint64_t n,
                            uint64_t* keys_out, void* vals_out)
{
    /* Sorting by (key as a 128-bit unsigned number, i) puts equal keys
     * together, keeps their input order (stability) and orders the groups by
     * key, so the result is unique. */
    if (n == 0) return 0;
    wki_t* t = (wki_t*)malloc(n * sizeof(wki_t));
    if (!t) return -1;
    for (uint64_t i = 0; i < n; i++) {
        t[i].lo = keys[2 * i];
        t[i].hi = keys[2 * i + 1];
        t[i].i = i;
    }
    qsort(t, n, sizeof(wki_t), cmp_wki);
    for (uint64_t p = 0; p < n; p++) {
        keys_out[2 * p] = keys[2 * t[p].i];
        keys_out[2 * p + 1] = keys[2 * t[p].i + 1];
        store_val(vals_out, vb, p, load_val(vals, vb, t[p].i));
    }
    free(t);
    return 0;
}

typedef struct { uint64_t hi, lo, start, len; } wrun_t;

static int cmp_wrun(const void* a, const void* b)
{
    const wrun_t* x = (const wrun_t*)a;
    const wrun_t* y = (const wrun_t*)b;
    if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
    if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
    if (x->start != y->start) return x->start < y->start ? -1 : 1;
    return 0;
}

int64_t orc_canonicalize_equal_wide(const uint64_t* keys, const void* vals, uint32_t vb, uint64_t n,
                                    uint64_t* canon_keys, void* canon_vals)
{
    if (n == 0) return -1;
    uint64_t nruns = 1;
    for (uint64_t p = 1; p < n; p++)
        if (keys[2 * p] != keys[2 * p - 2] || keys[2 * p + 1] != keys[2 * p - 1]) nruns++;
    wrun_t* r = (wrun_t*)malloc(nruns * sizeof(wrun_t));
    if (!r) return -2;
    uint64_t j = 0, p = 0;
    while (p < n) {
        uint64_t q = p;
        while (q < n && keys[2 * q] == keys[2 * p] && keys[2 * q + 1] == keys[2 * p + 1]) q++;
        r[j].lo = keys[2 * p];
        r[j].hi = keys[2 * p + 1];
        r[j].start = p;
        r[j].len = q - p;
        j++;
        p = q;
    }
    qsort(r, nruns, sizeof(wrun_t), cmp_wrun);
    /* two runs of one key are neighbours after the sort; the later one is
     * where contiguity broke */
    int64_t bad = -1;
    for (uint64_t x = 1; x < nruns; x++) {
        if (r[x].lo == r[x - 1].lo && r[x].hi == r[x - 1].hi) {
            if (bad < 0 || (int64_t)r[x].start < bad) bad = (int64_t)r[x].start;
        }
    }
    if (bad >= 0) {
        free(r);
        return bad;
    }
    uint64_t o = 0;
    for (uint64_t x = 0; x < nruns; x++) {
        for (uint64_t y = 0; y < r[x].len; y++) {
            canon_keys[2 * o] = keys[2 * (r[x].start + y)];
            canon_keys[2 * o + 1] = keys[2 * (r[x].start + y) + 1];
            store_val(canon_vals, vb, o, load_val(vals, vb, r[x].start + y));
            o++;
        }
    }
    free(r);
    return -1;
}

int orc_stats(const uint64_t* keys, uint64_t n, double heavy_threshold,
              uint64_t* distinct, uint64_t* max_freq, uint64_t* heavy_records)
{
    *distinct = 0;
    *max_freq = 0;
    *heavy_records = 0;
    if (n == 0) return 0;
    uint64_t* s = (uint64_t*)malloc(n * sizeof(uint64_t));
    if (!s) return -1;
    memcpy(s, keys, n * sizeof(uint64_t));
    qsort(s, n, sizeof(uint64_t), cmp_u64);
    uint64_t p = 0;
    while (p < n) {
        uint64_t q = p;
        while (q < n && s[q] == s[p]) q++;
        uint64_t c = q - p;
        (*distinct)++;
        if (c > *max_freq) *max_freq = c;
        if ((double)c > heavy_threshold) *heavy_records += c;
        p = q;
    }
    free(s);
    return 0;
}

/* ---- one level of Algorithm 1 ----------------------------------------- */

uint32_t orc_sample_size(uint64_t len, uint32_t c)
{
    /* ceil(c ln n'), capped at n'/8 so that small subproblems are not sampled
     * almost entirely, and at 16384 */
    if (len < 2) return 0;
    uint64_t s = (uint64_t)ceil((double)c * log((double)len));
    if (s > len / 8) s = len / 8;
    if (s > 16384) s = 16384;
    return (uint32_t)s;
}

uint32_t orc_heavy_threshold(uint64_t len)
{
    if (len < 3) return 1;
    return (uint32_t)ceil(log((double)len));
}

uint64_t orc_sample_index(uint64_t seed, uint32_t level, uint64_t start, uint64_t len,
                          uint64_t i)
{
    /* Counter-based draw: the stream key depends on (seed, level, start) and
     * the i-th draw mixes the key with i.  The 64-bit draw r is mapped to
     * [0, len) as floor(r * len / 2^64). */
    const uint64_t golden = 0x9e3779b97f4a7c15ULL;
    uint64_t k0 = orc_splitmix_mix(seed + golden * ((uint64_t)level + 1));
    uint64_t k1 = orc_splitmix_mix(k0 ^ start);
    uint64_t r = orc_splitmix_mix(k1 + golden * (i + 1));
    return (uint64_t)(((unsigned __int128)r * len) >> 64);
}

static int g_cmp_mode;

static int cmp_by_hash(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    uint64_t hx = orc_hash(x, g_cmp_mode), hy = orc_hash(y, g_cmp_mode);
    if (hx != hy) return hx < hy ? -1 : 1;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int64_t orc_select_heavy(const uint64_t* sample_keys, uint32_t s, uint32_t tau,
                         int hash_mode, uint32_t max_heavy, uint64_t* heavy_keys)
{
    /* Count the occurrences of each distinct sampled key; a key seen at least
     * tau times is heavy (Section 3.1, Algorithm 1 Step 1).  Distinct keys are
     * visited in ascending (h(k), k) order, so ids follow that order.
     * The heavy table has room for max_heavy keys (the paper's table is
     * unbounded): when more keys reach tau, tau is raised to the smallest
     * value at which at most max_heavy keys reach it. */
    if (s == 0) return 0;
    uint64_t* t = (uint64_t*)malloc((uint64_t)s * sizeof(uint64_t));
    uint32_t* runlen = (uint32_t*)malloc((uint64_t)s * sizeof(uint32_t));
    if (!t || !runlen) {
        free(t);
        free(runlen);
        return -2;
    }
    memcpy(t, sample_keys, (uint64_t)s * sizeof(uint64_t));
    g_cmp_mode = hash_mode;
    qsort(t, s, sizeof(uint64_t), cmp_by_hash);
    /* run lengths, recorded at each run's first position */
    uint32_t p = 0;
    while (p < s) {
        uint32_t q = p;
        while (q < s && t[q] == t[p]) q++;
        runlen[p] = q - p;
        p = q;
    }
    uint32_t eff = tau < 1 ? 1 : tau;
    for (;;) {
        uint64_t reach = 0;
        for (p = 0; p < s; p += runlen[p])
            if (runlen[p] >= eff) reach++;
        if (reach <= max_heavy) break;
        eff++;
    }
    int64_t nh = 0;
    for (p = 0; p < s; p += runlen[p])
        if (runlen[p] >= eff) heavy_keys[nh++] = t[p];
    free(t);
    free(runlen);
    return nh;
}

/* Position of k in the heavy list (sorted by (h, k)), or -1. */
static int64_t heavy_find(const uint64_t* hk, uint32_t nh, uint64_t k, int mode)
{
    uint64_t hkey = orc_hash(k, mode);
    int64_t lo = 0, hi = (int64_t)nh - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        uint64_t hm = orc_hash(hk[mid], mode);
        if (hm == hkey && hk[mid] == k) return mid;
        if (hm < hkey || (hm == hkey && hk[mid] < k)) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

void orc_bucket_ids(const uint64_t* keys, uint64_t n, const uint64_t* heavy_keys,
                    uint32_t n_heavy, uint32_t nl_bits, uint32_t shift, int hash_mode,
                    uint32_t* bids)
{
    const uint32_t n_light = 1u << nl_bits;
    for (uint64_t j = 0; j < n; j++) {
        int64_t pos = heavy_find(heavy_keys, n_heavy, keys[j], hash_mode);
        if (pos >= 0) {
            bids[j] = n_light + (uint32_t)pos;
        } else {
            uint64_t h = orc_hash(keys[j], hash_mode);
            bids[j] = (uint32_t)((h >> shift) & (uint64_t)(n_light - 1));
        }
    }
}

void orc_count_matrix(const uint32_t* bids, uint64_t n, uint64_t l, uint32_t nb,
                      uint32_t* C)
{
    uint64_t tiles = (n + l - 1) / l;
    memset(C, 0, tiles * nb * sizeof(uint32_t));
    for (uint64_t i = 0; i < tiles; i++) {
        uint64_t end = (i + 1) * l < n ? (i + 1) * l : n;
        for (uint64_t j = i * l; j < end; j++) C[i * nb + bids[j]] += 1;
    }
}

void orc_column_prefix(const uint32_t* C, uint64_t tiles, uint32_t nb, uint64_t n,
                       uint32_t* X, uint64_t* offsets)
{
    /* Walk C in column-major order (bucket by bucket, subarrays in order
     * inside a bucket) and write the running sum before each cell. */
    uint64_t run = 0;
    for (uint32_t j = 0; j < nb; j++) {
        for (uint64_t i = 0; i < tiles; i++) {
            X[i * nb + j] = (uint32_t)run;
            run += C[i * nb + j];
        }
    }
    for (uint32_t j = 0; j < nb; j++) offsets[j] = tiles ? X[j] : 0;
    offsets[nb] = n;
}

void orc_distribute(const uint64_t* keys, const void* vals, uint32_t vb,
                    const uint32_t* bids, uint64_t n, uint64_t l, uint32_t nb,
                    const uint32_t* X, uint64_t* t_keys, void* t_vals)
{
    uint64_t tiles = (n + l - 1) / l;
    uint32_t* x = (uint32_t*)malloc(nb * sizeof(uint32_t));
    if (!x) return;
    for (uint64_t i = 0; i < tiles; i++) {
        memcpy(x, X + i * nb, nb * sizeof(uint32_t));
        uint64_t end = (i + 1) * l < n ? (i + 1) * l : n;
        for (uint64_t j = i * l; j < end; j++) {
            uint32_t id = bids[j];
            t_keys[x[id]] = keys[j];
            store_val(t_vals, vb, x[id], load_val(vals, vb, j));
            x[id] += 1;
        }
    }
    free(x);
}
