/*
 * oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded CPU reference for semisort, histogram and
 * collect-reduce as defined in Dong, Wu, Wang, Dhulipala, Gu and Sun,
 * "High-Performance and Flexible Parallel Algorithms for Semisort and Related
 * Problems" (SPAA 2023).  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may call this library.  It shares no code,
 * header, helper or constant table with the GPU library; everything here is
 * written from the paper's definitions and from the published definitions of
 * the two mixing functions it uses.
 *
 * All pointers are host pointers owned by the caller.  Functions that can fail
 * (only on allocation) return a negative value; nothing else is checked.
 */
#ifndef SEMISORT_ORACLE_H
#define SEMISORT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- hashing ---------------------------------------------------------- */

/* User hash h (Section 2.1 asks the user for a hash family on keys).
 * mode 0: the 64-bit finalizer published with MurmurHash3 (a bijection).
 * mode 1: identity, the paper's "-i" variants (Section 4.1, Flexible Interface). */
uint64_t orc_hash(uint64_t k, int hash_mode);

/* SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014), used as the
 * counter-based generator that picks sample positions. */
uint64_t orc_splitmix_mix(uint64_t z);

/* ---- plain definitions (Section 2.1) ---------------------------------- */

/* semisort by equality: equal keys contiguous, input order kept among equal
 * keys (stability, Section 2.2).  Canonical group order: ascending (h(k), k).
 * val_bytes is 4 or 8.  Returns 0, or -1 when out of memory. */
int orc_semisort_equal(const uint64_t* keys, const void* vals, uint32_t val_bytes,
                       uint64_t n, int hash_mode, uint64_t* keys_out, void* vals_out);

/* semisort by comparison with groups in ascending key order, stable:
 * exactly a stable sort by key. */
int orc_semisort_less(const uint64_t* keys, const void* vals, uint32_t val_bytes,
                      uint64_t n, uint64_t* keys_out, void* vals_out);

/* semisort by equality of 128-bit keys (Section 2.1: any key type with an
 * equality test).  keys holds 2n words, key j = (keys[2j] low, keys[2j + 1]
 * high); keys_out likewise.  Canonical group order: ascending key as a 128-bit
 * unsigned number.  Returns 0, or -1 when out of memory. */
int orc_semisort_equal_wide(const uint64_t* keys, const void* vals, uint32_t val_bytes,
                            uint64_t n, uint64_t* keys_out, void* vals_out);

/* Canonical form of a candidate semisort of 128-bit keys: its runs reordered by
 * ascending key.  Returns -1 when equal keys are contiguous, else the position
 * of the first run whose key also occurs in another run; -2 when out of memory. */
int64_t orc_canonicalize_equal_wide(const uint64_t* keys, const void* vals, uint32_t val_bytes,
                                    uint64_t n, uint64_t* canon_keys, void* canon_vals);

/* histogram: (unique key, occurrences), ascending keys.  Returns m or -1. */
int64_t orc_histogram(const uint64_t* keys, uint64_t n, uint64_t* out_keys,
                      uint64_t* out_counts);

/* collect-reduce with map = value and monoid (+ mod 2^64, 0): (unique key,
 * wrapping sum of its values), ascending keys.  Returns m or -1. */
int64_t orc_collect_reduce(const uint64_t* keys, const uint64_t* vals, uint64_t n,
                           uint64_t* out_keys, uint64_t* out_sums);

/* collect-reduce with map = value and the monoid `op` (Section 3.5): 0 = (+ mod
 * 2^64, 0), 1 = (min, 2^64 - 1), 2 = (max, 0), 3 = (xor, 0) on uint64; (unique
 * key, fold of its values), ascending keys; 4 = first and 5 = last (the
 * value of the key's first / last record in input order) and 6 = affine
 * (a value (a, b) = (high, low 32 bits) is t -> a t + b mod 2^32; the fold
 * applies the maps in input order) and 7 = mat2 (a value's 16-bit fields
 * from the low end are the entries (a, b; c, d) of a 2 x 2 matrix over the
 * integers mod 2^16; the fold is the product in input order) are
 * non-commutative, folded in input order.  Returns m, -1 when out of memory,
 * -2 for an unknown op. */
int64_t orc_collect_reduce_monoid(const uint64_t* keys, const uint64_t* vals, uint64_t n, int op,
                                  uint64_t* out_keys, uint64_t* out_vals);

/* Transpose of a directed graph in CSR (Section 5, graph transposing):
 * nv vertices, ne edges, offs[nv + 1], cols[ne] < nv.  out_offs[nv + 1] and
 * out_cols[ne] receive the transposed CSR, each vertex's in-neighbours in
 * input order.  Returns 0, -1 when out of memory, -2 for an invalid CSR. */
int orc_transpose_csr(uint64_t nv, uint64_t ne, const uint64_t* offs, const uint32_t* cols,
                      uint64_t* out_offs, uint32_t* out_cols);

/* Canonical form of a candidate semisort_= output: split it into maximal runs
 * of equal keys and order the runs by ascending (h(k), k).  Because a stable
 * semisort is unique up to the order of its groups, a correct output has the
 * same canonical form as orc_semisort_equal's result.  Returns -1 when equal
 * keys are contiguous, otherwise the position of the first run whose key
 * already had an earlier run (canonical buffers are then unspecified), or -2
 * when out of memory. */
int64_t orc_canonicalize_equal(const uint64_t* keys, const void* vals, uint32_t val_bytes,
                               uint64_t n, int hash_mode, uint64_t* canon_keys,
                               void* canon_vals);

/* Table 3 statistics: distinct keys, maximum frequency, and the number of
 * records whose key occurs more than heavy_threshold times (the "Heavy Freq."
 * column uses 500 log n).  Returns 0 or -1. */
int orc_stats(const uint64_t* keys, uint64_t n, double heavy_threshold,
              uint64_t* distinct, uint64_t* max_freq, uint64_t* heavy_records);

/* ---- one level of Algorithm 1, step by step ---------------------------- */

/* Step 1 sample size |S| = ceil(c * ln n') (Algorithm 1 and Section 3.6,
 * natural logarithm), capped at n'/8 and at 16384, and heavy threshold
 * ceil(ln n'). */
uint32_t orc_sample_size(uint64_t len, uint32_t c);
uint32_t orc_heavy_threshold(uint64_t len);

/* Position in [0, len) of the i-th sample of the subproblem that starts at
 * `start` on recursion level `level`, drawn with replacement. */
uint64_t orc_sample_index(uint64_t seed, uint32_t level, uint64_t start, uint64_t len,
                          uint64_t i);

/* Heavy keys: the distinct sampled keys seen at least tau times, in ascending
 * (h(k), k) order; their bucket ids are n_L, n_L+1, ... in that order.  When
 * more than max_heavy keys qualify, tau is raised to the least value at which
 * at most max_heavy do.  Returns n_H, or -2 when out of memory. */
int64_t orc_select_heavy(const uint64_t* sample_keys, uint32_t s, uint32_t tau,
                         int hash_mode, uint32_t max_heavy, uint64_t* heavy_keys);

/* GetBucketId of Algorithm 1: the heavy id when k is a heavy key, otherwise
 * the light id taken from nl_bits bits of h(k) starting at bit `shift`. */
void orc_bucket_ids(const uint64_t* keys, uint64_t n, const uint64_t* heavy_keys,
                    uint32_t n_heavy, uint32_t nl_bits, uint32_t shift, int hash_mode,
                    uint32_t* bids);

/* Counting matrix C[i][j]: records of subarray i (size l, last one short)
 * whose bucket is j.  C is row-major ceil(n/l) x nb. */
void orc_count_matrix(const uint32_t* bids, uint64_t n, uint64_t l, uint32_t nb,
                      uint32_t* C);

/* Column-major prefix X[i][j] = sum of C over buckets j' < j, plus bucket j in
 * subarrays i' < i; offsets[j] = X[0][j], offsets[nb] = n. */
void orc_column_prefix(const uint32_t* C, uint64_t tiles, uint32_t nb, uint64_t n,
                       uint32_t* X, uint64_t* offsets);

/* Distribution into T: each subarray in order, T[X[i][id]++] = A[j]. */
void orc_distribute(const uint64_t* keys, const void* vals, uint32_t val_bytes,
                    const uint32_t* bids, uint64_t n, uint64_t l, uint32_t nb,
                    const uint32_t* X, uint64_t* t_keys, void* t_vals);

#ifdef __cplusplus
}
#endif

#endif
