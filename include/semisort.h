/*
 * semisort.h -- C-ABI of libsemisort_hip.so, an MI355X (gfx950) implementation
 * of the semisort family of Dong, Wu, Wang, Dhulipala, Gu and Sun,
 * "High-Performance and Flexible Parallel Algorithms for Semisort and Related
 * Problems" (SPAA 2023).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Keys are uint64.  Values are uint32 or uint64 (val_bytes = 4 or 8).
 *   Arrays are structure-of-arrays: keys[n] and vals[n] side by side, each
 *   aligned to its element size.
 * - Every array pointer is a DEVICE pointer on the context's device, owned by
 *   the caller.  The library owns only its workspace (temporary array T,
 *   counting matrices, heavy tables, work lists), which it grows on demand
 *   and frees in ss_destroy.
 * - Calls are ordered on the context's HIP stream.  A call returns after its
 *   work is enqueued; it synchronizes the stream once per recursion level to
 *   size the next level's launches, so it is not capture-safe.  Results are
 *   ready when the stream is.
 * - Errors: SS_EINVAL for bad arguments (checked before anything is
 *   enqueued), SS_ENOMEM when the workspace cannot grow, SS_EHIP for a failed
 *   HIP call, SS_EDEVICE for a condition detected on the device.  A semisort
 *   call returns without waiting for its last level's kernels; a condition
 *   they raise is reported by ss_sync or by the next call on the context.
 *   ss_last_error() returns a message for the last failure on the context.
 *   Nothing throws across the ABI.
 * - n = 0 is a no-op returning SS_OK.  n must be below 2^31 (positions are
 *   31-bit on the device).
 * - Output arrays must not overlap the inputs, except that keys_out == keys
 *   together with vals_out == vals is allowed for semisort (the paper's
 *   in-place form, Section 3.4).
 * - Randomness (sample positions) comes from a counter-based generator keyed
 *   by ss_params.seed, so results are deterministic for a fixed seed
 *   (race-free and internally deterministic, Section 2.2).
 */
#ifndef SEMISORT_HIP_H
#define SEMISORT_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ss_ctx ss_ctx;

typedef enum {
    SS_OK = 0,
    SS_EINVAL = -1,
    SS_ENOMEM = -2,
    SS_EHIP = -3,
    SS_EDEVICE = -4
} ss_status;

/* User hash h of Section 2.1.  SS_HASH_MIX64 is the 64-bit MurmurHash3
 * finalizer (a bijection); SS_HASH_IDENTITY uses the key itself, the "-i"
 * variants of Section 4.1 (Flexible Interface). */
typedef enum { SS_HASH_MIX64 = 0, SS_HASH_IDENTITY = 1 } ss_hash_mode;

/* Tunable parameters (Table 1 and Section 3.6).  Zero fields take defaults. */
typedef struct {
    uint32_t n_light_log2; /* b, n_L = 2^b light buckets on the top level (1..10; default 10) */
    uint32_t base_case;    /* alpha: subproblems below this are finished in LDS (64..4096; default 4096) */
    uint32_t sample_mult;  /* c in |S| = ceil(c ln n') (1..4096; default 800, the paper uses 500);
                              |S| <= min(n'/8, 16384) */
    uint32_t tile_min;     /* smallest subarray size l in records (power of two, 8192..65536) */
    uint32_t tile_max;     /* largest subarray size l (power of two, tile_min..65536; default 0: for
                              semisort_= 32768 on the first level and 16384 below, for semisort_<
                              32768 on the first level and 65536 below, else 65536) */
    uint32_t hash_mode;    /* ss_hash_mode */
    uint32_t heavy_min;    /* tau: a key sampled at least tau times is heavy (default 3; 0 = ceil(ln n'),
                              the paper's rule).  At most 512 keys per subproblem are heavy: if more
                              reach tau, tau rises to the least value that leaves at most 512. */
    uint32_t temp_records; /* 0 (default): semisort holds an n-record temporary array T.  Otherwise,
                              when the output is not the input (keys_out != keys), the first level
                              writes every bucket to the output and the levels below refine their
                              subproblems in groups through a pool of this many records (raised to
                              the largest subproblem if that is longer), in place of T.  In-place
                              calls, the reductions and the capturable batch keep T. */
    uint64_t seed;         /* sampling seed */
} ss_params;

/* Fill *p with the defaults. */
ss_status ss_default_params(ss_params* p);

/* Operations (Section 2.1): semisort_= and semisort_< reorder records;
 * histogram and collect-reduce (Section 3.5) emit one pair per distinct key. */
typedef enum {
    SS_OP_SEMISORT_EQUAL = 0,
    SS_OP_SEMISORT_LESS = 1,
    SS_OP_HISTOGRAM = 2,
    SS_OP_COLLECT_REDUCE = 3
} ss_op;

/* Create a context on HIP device `device` issuing work on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  workspace_cap bounds the
 * device memory the context's workspace may hold (bytes; 0 = no bound): a
 * call whose workspace would grow past it fails with SS_ENOMEM before
 * anything is enqueued or freed, and the context stays usable.  The
 * workspace grows on demand (by half again its size when that fits under
 * the cap) and is freed by ss_destroy.  The context also holds a small
 * status word and a second stream (default priority) for key fills. */
ss_status ss_create(int device, void* hip_stream, size_t workspace_cap, ss_ctx** out);
ss_status ss_destroy(ss_ctx* ctx);
ss_status ss_set_stream(ss_ctx* ctx, void* hip_stream);
const char* ss_last_error(ss_ctx* ctx);
/* Wait for the context's stream; SS_EDEVICE if a kernel of an earlier call
 * on the context raised a device condition that was not reported yet. */
ss_status ss_sync(ss_ctx* ctx);
/* Bytes of workspace the context holds now. */
ss_status ss_workspace_held(ss_ctx* ctx, size_t* bytes);
/* Planning query (no context, no device): an upper bound of the workspace
 * one call of operation `op` on n records makes a new context hold, for
 * val_bytes 4 or 8 (semisort; histogram and collect-reduce use 8) and the
 * given parameters (NULL = defaults).  A context created with workspace_cap
 * at least this value cannot fail that call with SS_ENOMEM because of the
 * cap.  The bound assumes the worst case of every level list (every
 * subproblem at the base-case size, one job per bucket): about 70 bytes per
 * record with the defaults, against about 22 actually held for the paper's
 * distributions.  It covers collect-reduce with the commutative monoids and
 * the ordered forms; the first/last monoids add 8 bytes per record and the
 * affine fold 16.  SS_EINVAL for an unknown op, a bad val_bytes or
 * parameters, or n >= 2^31. */
ss_status ss_workspace_bytes(int op, uint64_t n, uint32_t val_bytes, const ss_params* params,
                             size_t* bytes);

/* Engine options (tuning knobs that are not part of ss_params).
 * SS_OPT_DIST_VARIANT selects the shape of the semisort distribution kernel:
 *   0: LDS-staged writes, 16 waves per block, 8192-record sub-tiles (default)
 *   1: LDS-staged writes, 8 waves per block, 4096-record sub-tiles
 *   2..5: direct writes from registers (8 waves / 4 per SIMD, 8 waves / 6,
 *         16 waves / 4, 4 waves with 16 records per lane / 6)
 * Every variant gives the same result.  Values outside 0..5: SS_EINVAL. */
/* SS_OPT_DEEP_SAMPLE_DIV (1..64, default 1): below level 0 the sample size is
 * ceil((c / div) ln n').  SS_OPT_NL_TARGET (0 or 10..100, default 0): the number of
 * light buckets of a subproblem is chosen so that light buckets hold about
 * base_case * target / 100 records; 0 takes 50 for hash buckets and 35 for
 * the splitter buckets of semisort_< (their sizes vary more). */
/* SS_OPT_TILE0 / SS_OPT_TILE_DEEP (0 or a power of two in [8192, 65536],
 * default 0): the largest subarray of the first level / of the deeper levels,
 * overriding tile_max of the call's parameters (0: tile_max applies). */
/* SS_OPT_FOLD_ROUND (a power of two in [1, 1024], default 1024): the in-order
 * fold of SS_MONOID_AFFINE carries across 4096-record chunks in two levels,
 * 256 chunks per block and then the block totals in rounds of this many; a
 * smaller round exercises the cross-round carry on small inputs.  Every
 * value gives the same result. */
enum { SS_OPT_DIST_VARIANT = 1, SS_OPT_DEEP_SAMPLE_DIV = 2, SS_OPT_NL_TARGET = 3, SS_OPT_TILE0 = 4, SS_OPT_TILE_DEEP = 5,
       SS_OPT_FOLD_ROUND = 6 };
ss_status ss_set_option(ss_ctx* ctx, int option, int64_t value);

/* Kernel timing.  While enabled, every kernel launch of the engine is
 * bracketed by HIP events on the context's stream, grouped by pass:
 * SS_PROF_SAMPLE (Step 1; units = subproblems), SS_PROF_COUNT (counting pass;
 * units = records read), SS_PROF_SCAN (column-major prefix, four kernels;
 * units = subarrays), SS_PROF_DISTRIBUTE (distribution; units = records
 * moved), SS_PROF_PLAN (next-level planning and, for collect-reduce, the
 * heavy keys' results; units = subproblems), SS_PROF_FINISH (base cases and
 * copies; units = records), SS_PROF_COMPACT (packing of collect-reduce
 * and histogram results; units = positions scanned) and SS_PROF_FILL (keys of
 * one-key buckets written as constant runs; units = keys written; the
 * distribution pass does not store these keys).  ss_profile_enable
 * resets the totals; ss_profile_read waits for the stream and returns the
 * total milliseconds, launch count and units of one pass. */
enum {
    SS_PROF_SAMPLE = 0,
    SS_PROF_COUNT = 1,
    SS_PROF_SCAN = 2,
    SS_PROF_DISTRIBUTE = 3,
    SS_PROF_PLAN = 4,
    SS_PROF_FINISH = 5,
    SS_PROF_COMPACT = 6,
    SS_PROF_FILL = 7,
    SS_PROF_KINDS = 8
};
ss_status ss_profile_enable(ss_ctx* ctx, int on);
ss_status ss_profile_read(ss_ctx* ctx, int kind, double* total_ms, uint64_t* launches,
                          uint64_t* units);

/* semisort_= (Section 2.1; Algorithm 1 with the hash-table base case of
 * Section 3.3): reorders the n records so that equal keys are contiguous and
 * records with equal keys keep their input order (stable, Section 2.2).
 * The order of the groups is unspecified but deterministic for a seed.
 * params may be NULL (defaults). */
ss_status ss_semisort_equal(ss_ctx* ctx, const uint64_t* keys, const void* vals,
                            uint32_t val_bytes, uint64_t n, uint64_t* keys_out,
                            void* vals_out, const ss_params* params);

/* semisort_= and semisort_< (as ss_semisort_equal / ss_semisort_less) with
 * keys of key_bytes bytes (Section 2.1 defines the problem for any key type
 * with an equality test; Section 4.1 and the key-length study of Section 5
 * compare 32-, 64- and 128-bit keys): keys[n] and keys_out[n] hold
 * key_bytes-wide keys.
 *   4 or 8: unsigned integers.  A 32-bit key is hashed as its zero-extended
 *     64-bit value, so SS_HASH_MIX64 stays a bijection and the result equals
 *     the 64-bit call's on the zero-extended keys; its records move 4 bytes
 *     less per key through every pass.
 *   16: 128-bit keys, each two uint64 words, low word first, compared as whole
 *     keys (semisort_<: as 128-bit unsigned numbers); keys and keys_out
 *     16-byte aligned.
 *     SS_HASH_MIX64 hashes a key to 128 bits by a bijection (x = fmix64(low),
 *     then fmix64(high ^ x)); SS_HASH_IDENTITY uses the words themselves, low
 *     word first, which is slow when many keys share a low word (each level
 *     then separates few of them until the high word is reached).  A heavy
 *     bucket takes only records equal to one sampled key of its hash, so a
 *     colliding 64-bit level hash sends other keys to the light buckets.
 *     Workspace: beyond what ss_workspace_bytes reports for 8-byte keys, 8
 *     bytes more per record (temporary keys of 16 bytes) and 8 KB per
 *     subproblem of a level (the sampled key of every heavy id).
 *     semisort_< of 128-bit keys runs the stable semisort_= (the hash mode as
 *     given), numbers the runs of equal keys, sorts the m runs by key with two
 *     stable semisort_< passes over (word, run) pairs (low word, then high
 *     word) and scatters every record to its run's place; it holds the grouped
 *     records (n * (16 + val_bytes) bytes), a run-start bitmap (n / 8 bytes)
 *     and about 48 bytes per run besides the semisorts' own workspace, and waits
 *     once for m.
 * SS_EINVAL for another key_bytes or a misaligned 16-byte key array;
 * otherwise the arguments, conventions and errors of the 64-bit calls (in
 * place: keys_out == keys and vals_out == vals). */
ss_status ss_semisort_equal_keys(ss_ctx* ctx, const void* keys, uint32_t key_bytes, const void* vals,
                                 uint32_t val_bytes, uint64_t n, void* keys_out, void* vals_out,
                                 const ss_params* params);
ss_status ss_semisort_less_keys(ss_ctx* ctx, const void* keys, uint32_t key_bytes, const void* vals,
                                uint32_t val_bytes, uint64_t n, void* keys_out, void* vals_out,
                                const ss_params* params);

/* Batched semisort_=: `nseg` independent instances packed back to back;
 * instance i occupies [seg_offsets[i], seg_offsets[i+1]) of keys/vals and of
 * the outputs.  seg_offsets is a HOST array of nseg+1 non-decreasing
 * uint64 with seg_offsets[0] = 0 and seg_offsets[nseg] = total n.  Each
 * instance's result is the one ss_semisort_equal gives for it alone. */
ss_status ss_semisort_equal_batch(ss_ctx* ctx, const uint64_t* keys, const void* vals,
                                  uint32_t val_bytes, const uint64_t* seg_offsets,
                                  uint64_t nseg, uint64_t* keys_out, void* vals_out,
                                  const ss_params* params);

/* Batched semisort_= sized entirely on the device, for callers that record
 * the call into a HIP graph (stream capture) and replay it.  Same result as
 * ss_semisort_equal_batch (each instance's result is the one
 * ss_semisort_equal gives for it alone), but:
 * - seg_offsets is a DEVICE array of nseg+1 uint64 (non-decreasing,
 *   seg_offsets[0] = 0, seg_offsets[nseg] = n) and n is passed by the caller;
 *   offsets that break this raise a device condition (SS_EDEVICE at ss_sync).
 * - The host never waits: the first level is planned by a kernel from the
 *   offsets, and every later level's kernels run as resident grids that read
 *   the level's subproblem, subarray and job counts from device memory, where
 *   the previous level's planning put them (the per-level syncs of the other
 *   entry points size launches instead).  Work is taken from device-side
 *   queues: subarrays by per-XCD counters, base-case jobs by a counter.
 *   Exactly max_levels levels of launches are enqueued (1..64); subproblems
 *   still left after them raise a device condition, reported by ss_sync.
 *   With the default n_light_log2, inputs below 2^31 records need two levels
 *   (three when keys escape the sample); a level with no work costs about
 *   0.1 ms (fifteen launches that find nothing to do).
 * - Buffers are sized for the worst case of n records and the parameters:
 *   up to (8 + val_bytes + 46) bytes per record (temporary array, bucket
 *   ids, job and key-fill lists) plus about 63 KB per possible subproblem
 *   (n / base_case + 1 of them).  A call that needs more workspace
 *   than the context holds allocates it, and therefore must not be under
 *   stream capture (SS_EINVAL if it is): make one uncaptured call with the
 *   same n, nseg, val_bytes and params first.  A captured graph keeps the
 *   workspace addresses of that moment; the context must not grow its
 *   workspace (a larger call of any kind) while the graph is replayed, and
 *   calls on the context must not overlap the replays.
 * - Keys of one-key buckets are filled on the context's second stream, forked
 *   from and joined back to the call's stream with events (so a capture
 *   records both); the subarray size follows tile_min/tile_max only.
 * Supports hash_mode, base_case, n_light_log2, sample_mult, heavy_min, tile_*
 * and seed like the other calls; in place (keys_out == keys, vals_out ==
 * vals) is allowed. */
ss_status ss_semisort_equal_batch_capturable(ss_ctx* ctx, const uint64_t* keys, const void* vals,
                                             uint32_t val_bytes, const uint64_t* seg_offsets,
                                             uint64_t nseg, uint64_t n, uint64_t* keys_out,
                                             void* vals_out, uint32_t max_levels,
                                             const ss_params* params);

/* For callers that cannot allocate device memory (code under stream capture
 * that must not depend on an earlier sizing call, tight serving loops,
 * harnesses that forbid hipMalloc): ss_semisort_equal_batch_capturable with
 * the whole workspace in a static device array of the library (64 MiB,
 * one copy per device, held by every device the library runs on until the
 * process ends; its address is looked up once per device in ss_create).  The
 * call allocates nothing: no hipMalloc, hipFree or allocating library
 * routine.  Arguments, result, device conditions and errors are those of
 * ss_semisort_equal_batch_capturable, except:
 * - The workspace needed by the call's worst case (about 50 bytes per record
 *   with the default parameters and 8-byte values, more with a smaller
 *   base_case or tile_min) must fit in the array, else SS_EINVAL with the
 *   bytes needed, before anything is enqueued.  With the default parameters
 *   batches of up to 2^20 records fit, with either value width.
 * - Every call on a device shares that device's array, which keeps the last
 *   call's contents (each call clears the counters it needs): calls that
 *   overlap on one device -- on two streams, two contexts or two threads --
 *   race and give wrong results.  Serialize them.
 * - A captured graph of this call needs no earlier uncaptured call. */
ss_status ss_semisort_equal_batch_noalloc(ss_ctx* ctx, const uint64_t* keys, const void* vals,
                                          uint32_t val_bytes, const uint64_t* seg_offsets,
                                          uint64_t nseg, uint64_t n, uint64_t* keys_out,
                                          void* vals_out, uint32_t max_levels,
                                          const ss_params* params);

/* Autotuner for batched semisort_=: runs the batch with every parameter set
 * of a fixed grid around the defaults (sample_mult in {500, 800}, heavy_min in
 * {0, 3}, n_light_log2 in {8, 10}, base_case in {2048, 4096}, tile_max in
 * {32768, 65536}), `reps` timed runs each (HIP events on the context's
 * stream, after one warm-up run), and returns the fastest set in *best and
 * its time per run in *best_ms (host).  The outputs are overwritten with the
 * batch's result.  Arguments as for ss_semisort_equal_batch, except that the
 * outputs may not be the inputs.  Waits for the stream before returning.
 * Every parameter set gives a correct result; only the time differs. */
ss_status ss_autotune_equal_batch(ss_ctx* ctx, const uint64_t* keys, const void* vals,
                                  uint32_t val_bytes, const uint64_t* seg_offsets, uint64_t nseg,
                                  uint64_t* keys_out, void* vals_out, uint32_t reps,
                                  ss_params* best, double* best_ms);

/* Batched semisort_= with cached tuned parameters: the batch's class (key and
 * value widths, and the binary orders of its total size and of its mean
 * instance size) selects parameters the context tuned before; on the first
 * batch of a class, ss_autotune_equal_batch (one timed run per candidate)
 * picks them and the context keeps them.  Either way the outputs hold the
 * batch's result; *used receives the parameters and *tuned_now 1 when this
 * call tuned (both may be NULL).  Arguments as for ss_autotune_equal_batch.
 * ss_autotune_cache: with clear != 0 forgets every class; *entries receives
 * the number of classes kept (may be NULL). */
ss_status ss_semisort_equal_batch_tuned(ss_ctx* ctx, const uint64_t* keys, const void* vals,
                                        uint32_t val_bytes, const uint64_t* seg_offsets, uint64_t nseg,
                                        uint64_t* keys_out, void* vals_out, ss_params* used,
                                        int* tuned_now);
ss_status ss_autotune_cache(ss_ctx* ctx, int clear, uint64_t* entries);

/* semisort_< (Section 2.1 with the comparison base case of Section 3.3):
 * reorders the records into ascending key order, records with equal keys in
 * input order (stable).  The result is unique: a stable sort by key.
 * Buckets come from sorted splitters instead of hash bits (keys sampled
 * often enough get their own equality buckets, placed in key order), so the
 * concatenated buckets are already in key order; hash_mode is ignored.
 * params may be NULL (defaults). */
ss_status ss_semisort_less(ss_ctx* ctx, const uint64_t* keys, const void* vals,
                           uint32_t val_bytes, uint64_t n, uint64_t* keys_out,
                           void* vals_out, const ss_params* params);

/* Batched semisort_<: packed instances as in ss_semisort_equal_batch. */
ss_status ss_semisort_less_batch(ss_ctx* ctx, const uint64_t* keys, const void* vals,
                                 uint32_t val_bytes, const uint64_t* seg_offsets,
                                 uint64_t nseg, uint64_t* keys_out, void* vals_out,
                                 const ss_params* params);

/* One level of Algorithm 1 on one subproblem, for inspection: Step 1
 * (sampling, heavy keys, heavy table) and Step 2 (counting matrix, column-major
 * prefix, distribution), without Step 3.  Writes the distributed array T to
 * keys_out/vals_out, the n_L + n_H + 1 bucket offsets to offsets_out (device,
 * uint64, capacity 2^n_light_log2 + 512 + 1), the heavy keys' hashes in
 * bucket-id order to heavy_hashes_out (device, capacity 512) and n_H to
 * *n_heavy_out (host).  Light bucket ids use hash bits [0, n_light_log2). */
ss_status ss_partition_equal(ss_ctx* ctx, const uint64_t* keys, const void* vals,
                             uint32_t val_bytes, uint64_t n, uint64_t* keys_out,
                             void* vals_out, uint64_t* offsets_out,
                             uint64_t* heavy_hashes_out, uint32_t* n_heavy_out,
                             const ss_params* params);

/* collect-reduce (Section 3.5) with map = the record's value and the monoid
 * (+ mod 2^64, 0): for each distinct key k, the wrapping sum of the values of
 * the records with key k.  Heavy keys are reduced while their level is
 * distributed (their records are never moved); light buckets recurse as in
 * semisort_= and are reduced in LDS.  keys and vals are device arrays of n
 * uint64; out_keys and out_sums are device arrays with room for n entries
 * (the number m of distinct keys is not known in advance) that receive the m
 * pairs in an unspecified order that is deterministic for a seed; *m_out
 * (host) receives m.  The call waits for its stream before returning.
 * Outputs must not overlap the inputs or each other.  hash_mode selects the
 * user hash as for semisort_= (both are bijections, so a bucket in which all
 * 64 hash bits are used holds one key). */
ss_status ss_collect_reduce(ss_ctx* ctx, const uint64_t* keys, const uint64_t* vals,
                            uint64_t n, uint64_t* out_keys, uint64_t* out_sums,
                            uint64_t* m_out, const ss_params* params);

/* collect-reduce with another monoid (Section 3.5 defines collect-reduce for
 * any monoid (+, I), and notes that a stable algorithm needs no
 * commutativity): op selects it on uint64 values.  SS_MONOID_FIRST / _LAST
 * are non-commutative: each key's value is that of its first / last record
 * in input order (the positions are reduced with min / max and the values
 * fetched; n more uint64 of workspace).  SS_MONOID_AFFINE is a general
 * non-commutative fold: a stable semisort_= groups the records in input
 * order and a segmented scan folds each group (2n uint64 of workspace).  ordered = 0 gives the
 * pairs in an unspecified order (as ss_collect_reduce), 1 in ascending key
 * order (as ss_collect_reduce_ordered).  SS_MONOID_SUM is ss_collect_reduce
 * itself.  An op outside the enum: SS_EINVAL.  Otherwise the arguments,
 * conventions and errors of ss_collect_reduce. */
typedef enum {
    SS_MONOID_SUM = 0, /* (+ mod 2^64, 0) */
    SS_MONOID_MIN = 1, /* (min, 2^64 - 1) */
    SS_MONOID_MAX = 2, /* (max, 0) */
    SS_MONOID_XOR = 3, /* (xor, 0) */
    SS_MONOID_FIRST = 4, /* x (+) y = x, in input order */
    SS_MONOID_LAST = 5,  /* x (+) y = y, in input order */
    SS_MONOID_AFFINE = 6 /* composition of t -> a t + b mod 2^32, (a, b) the value's high and low
                            halves, applied in input order; identity (1, 0) */
} ss_monoid;
ss_status ss_collect_reduce_monoid(ss_ctx* ctx, const uint64_t* keys, const uint64_t* vals,
                                   uint64_t n, int op, int ordered, uint64_t* out_keys,
                                   uint64_t* out_vals, uint64_t* m_out, const ss_params* params);

/* collect-reduce with a caller's monoid (Section 3.5 defines collect-reduce for
 * any map and monoid; a stable semisort_= lets the fold run in input order, so
 * the operation need not be commutative).  ss_monoid_compile compiles, with
 * hipRTC for gfx950 and the context's device, a source text that defines
 *   ss_t                              the element type: trivially copyable, at
 *                                     most 8 bytes
 *   __device__ ss_t ss_identity()     the identity element
 *   __device__ ss_t ss_map(ss_u64 v)  the element of a record's value (its bits,
 *                                     zero-extended from val_bytes)
 *   __device__ ss_t ss_combine(ss_t a, ss_t b)   associative; a comes first in
 *                                     input order
 * (ss_u64 / ss_u32 / ss_u8 are defined before the source), into the kernels of
 * an in-order segmented fold.  The handle belongs to the caller and serves
 * calls on contexts of that device until ss_monoid_destroy.  A source that does
 * not compile gives SS_EINVAL with the compiler's messages in ss_last_error
 * (lines counted from 1 in the caller's text); compiling takes a fraction of a
 * second.
 * ss_collect_reduce_user: (unique key, fold of map(value) over its records in
 * input order) for the n records (keys uint64, vals val_bytes = 4 or 8 bytes
 * each); out_vals[i] holds the element's bytes zero-extended to 8.  Pairs in
 * an unspecified order, or ascending keys with ordered != 0.  Workspace: the
 * semisort's, plus 2n uint64 of fold results and n bytes of flags.  Other
 * conventions as ss_collect_reduce; SS_EINVAL for a handle of another device. */
typedef struct ss_user_monoid ss_user_monoid;
ss_status ss_monoid_compile(ss_ctx* ctx, const char* source, ss_user_monoid** out);
ss_status ss_monoid_destroy(ss_user_monoid* monoid);
ss_status ss_collect_reduce_user(ss_ctx* ctx, const ss_user_monoid* monoid, const uint64_t* keys,
                                 const void* vals, uint32_t val_bytes, uint64_t n, int ordered,
                                 uint64_t* out_keys, uint64_t* out_vals, uint64_t* m_out,
                                 const ss_params* params);

/* histogram (Section 3.5): collect-reduce with every value 1, so no value
 * array is read or moved.  out_counts[i] is the number of records with key
 * out_keys[i].  Same conventions as ss_collect_reduce. */
ss_status ss_histogram(ss_ctx* ctx, const uint64_t* keys, uint64_t n, uint64_t* out_keys,
                       uint64_t* out_counts, uint64_t* m_out, const ss_params* params);

/* Ordered forms: the same m pairs as ss_collect_reduce / ss_histogram, in
 * ascending key order (the order that semisort_< gives the groups, Section 3.4;
 * the sorted output of a group-by).  The unordered call runs first, then its
 * m pairs are sorted in place by the semisort_< path, so the extra work is
 * proportional to m, not n; params apply to both parts (hash_mode to the
 * first only).  Same arguments, conventions and errors as the unordered
 * calls; the call waits for its stream before returning. */
ss_status ss_collect_reduce_ordered(ss_ctx* ctx, const uint64_t* keys, const uint64_t* vals,
                                    uint64_t n, uint64_t* out_keys, uint64_t* out_sums,
                                    uint64_t* m_out, const ss_params* params);
ss_status ss_histogram_ordered(ss_ctx* ctx, const uint64_t* keys, uint64_t n, uint64_t* out_keys,
                               uint64_t* out_counts, uint64_t* m_out, const ss_params* params);

/* Forms of ss_collect_reduce_monoid and ss_histogram that leave m on the
 * device (Section 3.5; the count of distinct keys is known only at the end):
 * d_m is a DEVICE pointer to one uint64 that receives m, written on the
 * context's stream, and the call does not wait for its last kernels (its
 * levels still wait once each to size the next level's launches, as
 * semisort does).  With ordered = 1 the call reads m back once to size the
 * ordering of the pairs, then waits as the ordered forms do.  Arguments,
 * results and errors otherwise as the monoid / histogram calls; n = 0
 * writes m = 0. */
ss_status ss_collect_reduce_async(ss_ctx* ctx, const uint64_t* keys, const uint64_t* vals, uint64_t n,
                                  int op, int ordered, uint64_t* out_keys, uint64_t* out_vals,
                                  uint64_t* d_m, const ss_params* params);
ss_status ss_histogram_async(ss_ctx* ctx, const uint64_t* keys, uint64_t n, int ordered,
                             uint64_t* out_keys, uint64_t* out_counts, uint64_t* d_m,
                             const ss_params* params);

/* A batch of independent jobs of mixed operations (Section 2.1 and 3.5 for
 * each; thousands of small group-by instances in one call).  Every job gets
 * the result the single call gives for it alone: semisort_= as
 * ss_semisort_equal, semisort_< as ss_semisort_less, histogram as
 * ss_histogram_async (unordered) and collect-reduce as ss_collect_reduce_async
 * with the (+ mod 2^64, 0) monoid (unordered); m of a histogram or
 * collect-reduce job goes to its d_m (device).  Jobs are grouped by
 * operation and value width; in each group the jobs of at most
 * SS_BATCH_PACK_MAX records are gathered into one packed array by one kernel,
 * run as one batched call (one launch chain per level for all of them) and
 * their results scattered back by one kernel; larger jobs run one by one on
 * their own arrays.  Packing takes 4 x (8 + value bytes) bytes of workspace
 * per packed record (inputs and outputs, packed) besides the group's own.
 * Jobs may share inputs; no output may overlap another job's arrays or its
 * own inputs (in-place is not offered here).  SS_EINVAL for a bad job (op,
 * val_bytes, n >= 2^31, a null pointer, an overlap) before anything is
 * enqueued.  The call returns once everything is enqueued; results are
 * ready when the stream is (ss_sync reports device conditions).  params
 * apply to every job (NULL = defaults). */
enum { SS_BATCH_PACK_MAX = 1 << 22 };
typedef struct {
    int32_t op;          /* ss_op */
    uint32_t val_bytes;  /* 4 or 8 for semisort; ignored otherwise (collect-reduce values are u64) */
    uint64_t n;
    const uint64_t* keys;
    const void* vals;    /* unused by the histogram */
    void* out_a;         /* keys_out / out_keys: n entries */
    void* out_b;         /* vals_out / out_sums / out_counts: n entries */
    uint64_t* d_m;       /* histogram / collect-reduce: device uint64 receiving m; unused by semisort */
} ss_job;
ss_status ss_batch(ss_ctx* ctx, const ss_job* jobs, uint64_t njobs, const ss_params* params);

/* Transpose of a directed graph in CSR (Section 5, graph transposing): the
 * transpose holds (u, v) for every edge (v, u), which for a CSR input is a
 * semisort of the edges by their other endpoint; a stable one keeps every
 * vertex's new neighbours in input order (ascending for a row-ordered CSR).
 * nv vertices (below 2^32), ne edges (below 2^31); offsets[nv + 1] (uint64,
 * non-decreasing from 0 to ne) and cols[ne] (uint32 targets below nv) are
 * device arrays of the input; out_offsets[nv + 1] and out_cols[ne] receive the
 * transpose.  The edges are expanded to (target, source) records, sorted by
 * the semisort_< path (stable), and the new offsets are the first position of
 * every target (vertices without edges take the next one).  Workspace: 20
 * bytes per edge besides semisort_<'s own.  SS_EINVAL for bad sizes,
 * overlapping arrays or offsets that do not start at 0 and end at ne (read
 * once from the device); SS_EDEVICE when an offset decreases or a target is
 * not below nv.  The call waits for its stream before returning. */
ss_status ss_transpose_csr(ss_ctx* ctx, uint64_t nv, uint64_t ne, const uint64_t* offsets,
                           const uint32_t* cols, uint64_t* out_offsets, uint32_t* out_cols,
                           const ss_params* params);

/* ---- serving (continuous batching of group-by requests) ----------------
 *
 * A server owns `lanes` worker threads, each driving its own context on its
 * own HIP stream (default priority), so requests on different lanes overlap
 * on the device.  Requests wait in arrival order; a free lane takes the
 * oldest request that fits in hbm_budget together with everything else being
 * served, and the requests of at most pack_max_records records waiting
 * behind it -- of any operation -- join the same call, up to batch_records
 * records and 4096 requests: the lane runs them as one ss_batch (packed
 * into one launch chain per operation and level).  Every request gets the
 * result it gets alone.  The budget counts the arrays of the requests being
 * served (inputs and outputs) and each lane's workspace: what its context
 * holds plus the planning bound (ss_workspace_bytes) of what the call may
 * add; an idle lane gives its workspace back when nothing else fits.
 * Inputs and outputs are caller-owned device arrays that must stay valid
 * until the request is done.  Completion is taken on the host once the
 * lane's stream has drained; latency runs from the arrival time to then. */
typedef struct {
    int32_t op;          /* ss_op */
    uint32_t val_bytes;  /* 4 or 8 for semisort; ignored otherwise (collect-reduce values are u64) */
    uint64_t n;
    const uint64_t* keys;
    const void* vals;    /* unused by the histogram */
    void* out_a;         /* keys_out / out_keys, n entries */
    void* out_b;         /* vals_out / out_sums / out_counts, n entries */
} ss_request;

typedef struct {
    uint32_t lanes;             /* 1..16 (default 4) */
    uint32_t pack_max_records;  /* largest request that joins another's call (default 2^20; 0 = never) */
    uint64_t batch_records;     /* most records of one packed call (default 2^24) */
    uint64_t hbm_budget;        /* bytes of device memory the requests being served and the lanes'
                                   workspace may hold (default 200 GiB) */
    ss_params params;           /* parameters of every call (default ss_default_params) */
} ss_server_config;

typedef struct ss_server ss_server;

ss_status ss_server_default_config(ss_server_config* cfg);
/* cfg may be NULL (defaults).  SS_EINVAL for a bad device or lane count. */
ss_status ss_server_create(int device, const ss_server_config* cfg, ss_server** out);
/* Seconds since the server was created (the clock of arrival times). */
double ss_server_now(ss_server* srv);
/* Queue a request (does not block on the device).  arrival_s: its arrival on
 * the server clock, or <= 0 for now.  *ticket identifies it in ss_server_poll.
 * SS_EINVAL for a malformed request, SS_ENOMEM for one whose arrays and
 * workspace bound can never fit in the budget.  Inputs must be complete on
 * the device: the lanes do not wait for other streams. */
ss_status ss_server_submit(ss_server* srv, const ss_request* req, double arrival_s, uint64_t* ticket);
/* *done = 1 once the request is complete; then *result is its status,
 * *latency_s its latency and *m its group count (histogram and collect-reduce).
 * result, latency_s and m may be NULL.  SS_EINVAL for an unknown ticket. */
ss_status ss_server_poll(ss_server* srv, uint64_t ticket, int* done, ss_status* result,
                         double* latency_s, uint64_t* m);
/* Wait until every submitted request is complete. */
ss_status ss_server_drain(ss_server* srv);
/* Requests completed, device calls made, requests that were packed with
 * others, and the largest device memory the server reserved (bytes; never
 * above the budget). */
ss_status ss_server_stats(ss_server* srv, uint64_t* completed, uint64_t* calls, uint64_t* packed,
                          uint64_t* peak_reserved);
/* Stop the lanes and free everything; requests still waiting are dropped
 * (drain first). */
ss_status ss_server_destroy(ss_server* srv);

#ifdef __cplusplus
}
#endif

#endif
