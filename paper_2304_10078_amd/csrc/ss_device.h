// Device side of the semisort engine: data structures, wave primitives and the
// kernels of one recursion level (Algorithm 1 of Dong et al., SPAA 2023),
// written for gfx950 (CDNA4, wave64, 160 KB LDS per CU).
//
// Layout conventions
//   * keys[] (u32, u64 or 128-bit) and vals[] (u32 or u64) are separate
//     arrays (SoA).  In registers a key of up to 64 bits is held zero-extended
//     to 64 bits; a 128-bit key as its two words.
//   * A recursion level holds a list of subproblems (Seg).  Every kernel of
//     the level runs over all of them at once: a block finds its subproblem
//     by binary search over the subproblems' first tile / chunk.
//   * The counting matrix of Section 3.2 is stored one row per subarray
//     ("tile"), row stride kNbStride u32, and is overwritten in place by the
//     column-major prefix X (absolute output positions).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace ssd {

constexpr uint32_t kHeavyMax = 512;          // n_H cap per subproblem
constexpr uint32_t kLightBitsMax = 10;       // n_L <= 2^10
constexpr uint32_t kNbStride = (1u << kLightBitsMax) + kHeavyMax;  // 1536 buckets max
constexpr uint32_t kSampleMax = 16384;       // |S| cap (LDS bitonic capacity)
constexpr uint32_t kHeavySlotsMax = 1024;    // slots per heavy table; two tables (load <= 1/4)
constexpr uint32_t kAlphaMax = 4096;         // largest base case held in LDS
constexpr uint32_t kChunk = 32;              // subarrays per scan chunk
constexpr uint32_t kCopyChunk = 65536;       // records per copy job
constexpr uint32_t kFillChunk = 262144;      // records per key-fill job
constexpr uint32_t kBucketGroups = kNbStride / 64;  // 24 column groups in the bucket scan
constexpr uint16_t kEmpty16 = 0xFFFF;
constexpr uint32_t kEmpty32 = 0xFFFFFFFFu;

// device status bits
constexpr uint32_t kStatusSizeMismatch = 1u;   // bucket sizes do not add up to the subproblem
constexpr uint32_t kStatusScatterRange = 2u;   // a distribution target fell outside its subproblem
constexpr uint32_t kStatusBaseIndex = 4u;      // a base-case permutation entry out of range
constexpr uint32_t kStatusHeavyTable = 8u;     // the heavy table could not be built
constexpr uint32_t kStatusBadOffsets = 16u;    // instance offsets not non-decreasing from 0 to n
constexpr uint32_t kStatusTooDeep = 32u;       // subproblems left after the last device-sized level
constexpr uint32_t kStatusCapacity = 64u;      // a device-sized level outgrew a reserved list
constexpr uint32_t kStatusBadGraph = 128u;     // CSR offsets not non-decreasing, or a target >= the vertex count

struct Seg {
    uint32_t start;    // absolute first record
    uint32_t len;
    uint32_t ibase;    // first record of the instance the subproblem belongs to
    uint32_t tile0;    // first tile of the subproblem in the level's tile list
    uint32_t chunk0;   // first scan chunk
    uint32_t ntiles;
    uint8_t nl_bits;   // light id bits b (n_L = 2^b); a cap until the sampling kernel refines it
    uint8_t shift;     // first hash bit of the light id (hash-bucketed subproblems)
    uint16_t nbk;      // number of buckets, written by the sampling kernel
    uint16_t nheavy;   // n_H, written by the sampling kernel
    uint16_t hlog2;    // bits 0-7: log2 slots per heavy table (0 when n_H = 0); bits 8-14: table salt;
                       // bit 15: slots read directly from the hash (heavy_slot)
};
static_assert(sizeof(Seg) == 32, "Seg layout");

struct Job {
    uint32_t start;
    uint32_t len;
};

// Monoids of collect-reduce on uint64 values (Section 3.5 allows any monoid):
// 0 = (+ mod 2^64, 0), 1 = (min, 2^64 - 1), 2 = (max, 0), 3 = (xor, 0).  All
// are commutative, so partial results may be combined in any order (LDS and
// global atomics).  op is uniform across a launch.
__device__ __forceinline__ unsigned long long red_identity(uint32_t op)
{
    return op == 1 ? ~0ull : 0ull;
}

__device__ __forceinline__ unsigned long long red_combine(uint32_t op, unsigned long long x, unsigned long long y)
{
    return op == 0 ? x + y : op == 1 ? (x < y ? x : y) : op == 2 ? (x > y ? x : y) : x ^ y;
}

__device__ __forceinline__ void red_atomic(uint32_t op, unsigned long long* p, unsigned long long v)
{
    switch (op) {
    case 0: atomicAdd(p, v); break;
    case 1: atomicMin(p, v); break;
    case 2: atomicMax(p, v); break;
    default: atomicXor(p, v); break;
    }
}

// Keys of a one-key final bucket, written as a constant run instead of being
// moved record by record.
struct FillJob {
    uint32_t start;
    uint32_t len;
    uint64_t key;
};

// Job classes: base cases by capacity (512, 1024, 2048, 4096 records), then copies.
constexpr int kJobClasses = 5;
constexpr int kCopyClass = 4;

__host__ __device__ __forceinline__ int base_class(uint32_t len)
{
    return len <= 512 ? 0 : len <= 1024 ? 1 : len <= 2048 ? 2 : 3;
}

struct LevelInfo {
    uint32_t nsegs;                  // subproblems emitted for the next level
    uint32_t njobs[kJobClasses];     // jobs emitted by this level, per class
    uint32_t nfills;                 // key-fill jobs emitted by this level
    uint32_t tiles;                  // tiles of the next level
    uint32_t chunks;                 // scan chunks of the next level
    uint32_t tile;                   // subarray size of the next level
    uint32_t status;                 // device-detected errors
    unsigned long long records;      // records in the next level's subproblems
    unsigned long long job_records;  // records covered by this level's jobs
    unsigned long long fill_records; // records whose keys this level's fill jobs write
    uint32_t smp_total;              // sample size of subproblem 0 of the last sampled level
    uint32_t smp_heavy;              // of those, samples of heavy keys
};

struct LevelArgs {
    const uint64_t* src_keys;
    const void* src_vals;
    uint64_t* dst_keys;    // destination of buckets that need more work
    void* dst_vals;
    uint64_t* fin_keys;    // destination of buckets that are final (may equal dst)
    void* fin_vals;
    uint16_t* bids;        // bucket id of every record, written by the counting pass
    uint64_t* sink;        // 512 bytes that absorb the stores of lanes without a record
    Seg* segs;
    uint32_t nsegs;
    uint32_t tile;
    uint32_t* C;           // [tiles][kNbStride]
    uint32_t* P;           // [chunks][kNbStride]
    uint32_t* tot;         // [nsegs][kNbStride]
    uint32_t* bstart;      // [nsegs][kNbStride + 1]
    uint64_t* heavy_list;  // [nsegs][kHeavyMax]  heavy hashes in id order
    uint64_t* tab_h;       // [nsegs][2][kHeavySlotsMax]  two-choice heavy table
    uint16_t* tab_id;      // [nsegs][2][kHeavySlotsMax]
    LevelInfo* info;
    uint64_t seed;
    uint32_t level;
    uint32_t sample_mult;
    uint32_t heavy_min;    // heavy threshold tau; 0 = ceil(ln n')
    uint32_t deep_div;     // below level 0 the sample multiplier is divided by this
    uint32_t nl_target;    // adaptive n_L aims at light buckets of alpha * nl_target / 100 records
    uint32_t alpha;
    uint32_t adaptive_nl;  // choose n_L per subproblem from the sample's light fraction
    uint32_t ordered;      // buckets from sorted splitters (semisort_<) instead of hash bits
    uint8_t* bfin;         // [nsegs][kNbStride]: 1 for buckets that are final (one key each)
    uint64_t* bkey;        // [nsegs][kNbStride]: the key of each one-key bucket
    uint32_t* top;         // [nsegs]: the two most sampled heavy buckets (16 bits each, 0xFFFF = none)
    uint32_t fill_heavy;   // one-key buckets bound for keys_out: values move, keys are filled later
    // collect-reduce / histogram (Section 3.5)
    uint32_t reduce;                // heavy records are summed where they are, not moved
    unsigned long long* hsum;       // [nsegs][kHeavyMax] sums of heavy records per heavy id
    uint64_t* res_keys;             // results at position coordinates (n entries)
    uint64_t* res_vals;
    uint8_t* rflag;                 // 1 where a result sits
    uint32_t rop;                   // collect-reduce monoid (red_* below); histogram: 0
    // device-sized levels (the *_ds kernels): the level's subproblem, tile and
    // chunk counts and subarray size are read from dims, written there by the
    // previous level's planning; seg_cap bounds the subproblem list
    const LevelInfo* dims;
    uint32_t seg_cap;
    uint32_t* q;  // the level's work-queue counters, zero at the start: [0, 8) counting, [8, 16) distribution
    // 128-bit keys: one sampled key per heavy id ([nsegs][kHeavyMax] pairs of words)
    uint64_t* hrep;
};

// ---------------------------------------------------------------- hashing

// MurmurHash3's 64-bit finalizer (Appleby): a bijection on 64-bit words.
__device__ __forceinline__ uint64_t fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

template <int MODE>
__device__ __forceinline__ uint64_t user_hash(uint64_t k)
{
    if constexpr (MODE == 1) return k;
    else return fmix64(k);
}

// Inverse of fmix64: xor-shift by 33 undoes itself on 64-bit words, and the
// two multipliers are odd, so their inverses mod 2^64 exist.
__device__ __forceinline__ uint64_t unfmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0x9cb4b2f8129337dbULL;
    k ^= k >> 33;
    k *= 0x4f74430c22a54005ULL;
    k ^= k >> 33;
    return k;
}

template <int MODE>
__device__ __forceinline__ uint64_t key_of_hash(uint64_t h)
{
    if constexpr (MODE == 0) return unfmix64(h);
    else return h;
}


// ---------------------------------------------------------------- key types
// Keys of 4 and 8 bytes are handled as 64-bit words (a 4-byte key
// zero-extended); their hash is a bijection on 64 bits, so equal hashes mean
// equal keys.  A 128-bit key (two words, low word first in memory) is held as
// Key128; its hash is a bijection on 128 bits whose low word drives the first
// 64 bits of bucketing and heavy detection, and the high word the rest.  Its
// 64-bit level hash can collide, so heavy ids are confirmed against a sampled
// key and the base cases compare whole keys.

struct alignas(16) Key128 {
    uint64_t lo, hi;
};

__device__ __forceinline__ bool operator==(const Key128& a, const Key128& b) { return a.lo == b.lo && a.hi == b.hi; }

template <typename K> struct KeyTraits {
    using R = uint64_t;  // register form
    static constexpr uint32_t hash_bits = 64;
    static constexpr bool wide = false;
};
template <> struct KeyTraits<Key128> {
    using R = Key128;
    static constexpr uint32_t hash_bits = 128;
    static constexpr bool wide = true;
};
template <typename K> using KReg = typename KeyTraits<K>::R;
template <typename K> constexpr bool kWide = KeyTraits<K>::wide;

template <typename K>
__device__ __forceinline__ KReg<K> kload(const K* p)
{
    if constexpr (kWide<K>) return *p;
    else return (uint64_t)*p;
}

template <typename K>
__device__ __forceinline__ K knarrow(const KReg<K>& r)
{
    return (K)r;
}
template <>
__device__ __forceinline__ Key128 knarrow<Key128>(const Key128& r)
{
    return r;
}

// 64-bit fold of a key for LDS table slots (equal keys, equal folds).
__device__ __forceinline__ uint64_t kfold(uint64_t k) { return k; }
__device__ __forceinline__ uint64_t kfold(const Key128& k) { return k.lo ^ (k.hi * 0x9e3779b97f4a7c15ULL); }

// The two hash words of a key (hi is 0 for keys of up to 64 bits).
struct Hash2 {
    uint64_t lo, hi;
};

template <int MODE>
__device__ __forceinline__ Hash2 khash(uint64_t k)
{
    return Hash2{user_hash<MODE>(k), 0ull};
}

// 128-bit keys.  Identity (MODE 1): the key's own words.  Mixed: x = fmix64(lo)
// then y = fmix64(hi ^ x), hash (y, x); each step is invertible given the
// other word, so the map is a bijection on 128 bits, and y depends on every
// bit of the key.
template <int MODE>
__device__ __forceinline__ Hash2 khash(const Key128& k)
{
    if constexpr (MODE == 1) return Hash2{k.lo, k.hi};
    else {
        const uint64_t x = fmix64(k.lo);
        return Hash2{fmix64(k.hi ^ x), x};
    }
}

// Hash that identifies heavy keys at a level starting at hash bit `shift`:
// the word that holds the level's first bucket bit.
__device__ __forceinline__ uint64_t level_hash(const Hash2& h, uint32_t shift) { return shift < 64 ? h.lo : h.hi; }

// Hash bits from `shift` on, as a 64-bit window (shift < 128).
__device__ __forceinline__ uint64_t hash_window(const Hash2& h, uint32_t shift)
{
    if (shift == 0) return h.lo;
    if (shift < 64) return (h.lo >> shift) | (h.hi << (64 - shift));
    return h.hi >> (shift - 64);
}

// SplitMix64's output function (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// Table slot from a hash: fold to 32 bits and keep the top bits of the
// product with 2^32/phi (Fibonacci hashing), so identity-hashed small
// integers still spread; one 32-bit multiply.
__device__ __forceinline__ uint32_t fib_slot(uint64_t h, uint32_t log2slots)
{
    const uint32_t x = (uint32_t)h ^ (uint32_t)(h >> 32);
    return (x * 0x9e3779b1u) >> (32 - log2slots);
}

// Second slot of the two-choice heavy table: an independent 32-bit mix of
// the hash, perturbed by a per-table salt.
__device__ __forceinline__ uint32_t slot2(uint64_t h, uint32_t log2slots, uint32_t salt)
{
    const uint32_t x = ((uint32_t)(h >> 32) + salt * 0x632be5abu) * 0x85ebca6bu ^ (uint32_t)h * 0xc2b2ae35u;
    return x >> (32 - log2slots);
}

// Slots of the two-choice heavy table.  With a mixed hash and fewer than 32
// hash bits consumed by the levels above (bit 15 of the table field), the
// slots come from the hash directly: its top bits for the first table, one
// salted multiply of bits 16..47 for the second.  Otherwise (identity keys,
// very deep subproblems whose keys share many low bits) the hash is folded
// and mixed first.
constexpr uint32_t kDirectSlots = 0x8000u;

__device__ __forceinline__ uint32_t heavy_slot(uint64_t h, uint32_t hfield, int side)
{
    const uint32_t lg = hfield & 0xFFu, salt = (hfield >> 8) & 0x7Fu;
    if (hfield & kDirectSlots) {
        if (side == 0) return (uint32_t)(h >> 32) >> (32 - lg);
        return ((uint32_t)(h >> 16) * (0x85ebca6bu + 2u * salt)) >> (32 - lg);
    }
    return side == 0 ? fib_slot(h, lg) : slot2(h, lg, salt);
}

// GetBucketId (Algorithm 1): the heavy id when the key is in the heavy table,
// else the light id from nl_bits bits of the hash starting at `shift`.  The
// heavy table has two choices per key (cuckoo hashing), so a lookup is four
// independent LDS reads and no probe loop.  K: 0 = no heavy table, 1 = direct
// slots, 2 = mixed slots (the caller branches once per subproblem).
// `w` holds the hash bits from the level's first bucket bit on, `h` the level
// hash the heavy table is keyed by.
template <int K>
__device__ __forceinline__ uint32_t bucket_of_w(uint64_t h, uint64_t w, const uint64_t* th, const uint16_t* tid,
                                                uint32_t hfield, uint32_t lmask)
{
    uint32_t b = (uint32_t)w & lmask;
    if constexpr (K != 0) {
        const uint32_t s1 = heavy_slot(h, (hfield & 0x7FFFu) | (K == 1 ? kDirectSlots : 0u), 0);
        const uint32_t s2 = heavy_slot(h, (hfield & 0x7FFFu) | (K == 1 ? kDirectSlots : 0u), 1) + kHeavySlotsMax;
        const uint16_t i1 = tid[s1], i2 = tid[s2];
        const uint64_t h1 = th[s1], h2 = th[s2];
        if (i2 != kEmpty16 && h2 == h) b = i2;
        if (i1 != kEmpty16 && h1 == h) b = i1;
    }
    return b;
}

template <int K>
__device__ __forceinline__ uint32_t bucket_of(uint64_t h, const uint64_t* th, const uint16_t* tid,
                                              uint32_t hfield, uint32_t shift, uint32_t lmask)
{
    return bucket_of_w<K>(h, h >> shift, th, tid, hfield, lmask);
}

// ---------------------------------------------------------------- wave / block helpers

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of lanes below this one whose bit is set in m.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lanes of the wave whose value d equals mine (gfx950 has no match_any, so
// one ballot per bit).  All 64 lanes must be active; `live` masks out lanes
// that carry no record.
__device__ __forceinline__ uint64_t wave_match(uint32_t d, uint32_t nbits, uint64_t live)
{
    uint64_t peers = live;
    for (uint32_t bit = 0; bit < nbits; ++bit) {
        const bool x = (d >> bit) & 1u;
        const uint64_t bal = __ballot(x);
        peers &= x ? bal : ~bal;
    }
    return peers;
}

// Stable rank of this lane's record among the records of the wave's chunk
// processed so far with the same digit, using the wave's private counters
// wcw[digit].  Lanes are taken in lane order, rounds in program order.
__device__ __forceinline__ uint32_t wave_rank(uint32_t d, bool valid, uint32_t nbits, uint16_t* wcw)
{
    const uint64_t live = __ballot(valid);
    const uint64_t peers = wave_match(d, nbits, live);
    uint32_t r = 0;
    if (valid) {
        const uint32_t pre = wcw[d];
        const uint32_t below = lanes_below(peers);
        if (below == 0) wcw[d] = (uint16_t)(pre + __popcll(peers));
        r = pre + below;
    }
    __builtin_amdgcn_wave_barrier();
    return r;
}

constexpr int ilog2_c(uint32_t x) { return x <= 1 ? 0 : 1 + ilog2_c(x >> 1); }

// wave_rank for the E records a lane holds in one round, digits below 2^NB.
// The match masks come first, all E at once (their ballots are independent,
// so they interleave, and with the bit count fixed the loop unrolls); only
// the counter updates run in record order.  Bits above a digit's width are
// zero in every lane and leave the masks unchanged.
template <int E, int NB = 11>
__device__ __forceinline__ void wave_rank_all(const uint32_t (&d)[E], const bool (&valid)[E], uint32_t nbits,
                                              uint16_t* wcw, uint32_t (&r)[E])
{
    uint64_t peers[E];
    if (NB <= 8 || nbits > 6) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            uint32_t lo = 0, hi = 0;  // lanes whose digit differs in some bit
#pragma unroll
            for (int bit = 0; bit < NB; ++bit) {
                uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d[e], bit, 1);  // 0 or ~0
                // opaque to the optimizer, so that the ballot compares m itself
                // instead of recomputing the bit (one instruction less per bit)
                __asm__("" : "+v"(m));
                const uint64_t bal = __ballot(m != 0);
                // x | (m ^ bal) in one instruction (truth table over m, x, bal)
                lo = __builtin_amdgcn_bitop3_b32(m, lo, (uint32_t)bal, 0xDE);
                hi = __builtin_amdgcn_bitop3_b32(m, hi, (uint32_t)(bal >> 32), 0xDE);
            }
            peers[e] = __ballot(valid[e]) & ~(((uint64_t)hi << 32) | lo);
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) peers[e] = wave_match(d[e], nbits, __ballot(valid[e]));
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        uint32_t rr = 0;
        if (valid[e]) {
            const uint32_t pre = wcw[d[e]];
            const uint32_t below = lanes_below(peers[e]);
            if (below == 0) wcw[d[e]] = (uint16_t)(pre + __popcll(peers[e]));
            rr = pre + below;
        }
        __builtin_amdgcn_wave_barrier();
        r[e] = rr;
    }
}

// Exclusive scan over the block of one u32 per thread; tmp holds >= 17 u32.
template <int BS>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* tmp, uint32_t* total)
{
    constexpr int NW = BS / 64;
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63) tmp[w] = x;
    __syncthreads();
    if (w == 0) {
        uint32_t t = lane < (uint32_t)NW ? tmp[lane] : 0u;
#pragma unroll
        for (int o = 1; o < NW; o <<= 1) {
            uint32_t y = __shfl_up(t, o, 64);
            if (lane >= (uint32_t)o) t += y;
        }
        if (lane < (uint32_t)NW) tmp[lane] = t;
    }
    __syncthreads();
    const uint32_t base = w ? tmp[w - 1] : 0u;
    if (total) *total = tmp[NW - 1];
    __syncthreads();
    return base + x - v;
}

// Exclusive scan over the block of E values per thread taken as rows: value
// e of thread t stands for element e*BS + t, so ex[e] = (sum of all values of
// rows e' < e) + (sum of row e over threads t' < t).  tmp holds E*BS/64 + E
// u32.
template <int BS, int E>
__device__ __forceinline__ void block_excl_scan_rows(const uint32_t (&v)[E], uint32_t (&ex)[E], uint32_t* tmp)
{
    constexpr int NW = BS / 64;
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    uint32_t x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = v[e];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t y = __shfl_up(x[e], o, 64);
            if (lane >= (uint32_t)o) x[e] += y;
        }
    }
    if (lane == 63) {
#pragma unroll
        for (int e = 0; e < E; ++e) tmp[e * NW + w] = x[e];
    }
    __syncthreads();
    if (threadIdx.x < (uint32_t)E) {
        const uint32_t e = threadIdx.x;
        uint32_t run = 0;
        for (int ww = 0; ww < NW; ++ww) {
            const uint32_t t = tmp[e * NW + ww];
            tmp[e * NW + ww] = run;
            run += t;
        }
        tmp[E * NW + e] = run;  // row total
    }
    __syncthreads();
    uint32_t rowoff = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        ex[e] = rowoff + tmp[e * NW + w] + x[e] - v[e];
        rowoff += tmp[E * NW + e];
    }
    __syncthreads();
}

// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X.  Give
// each XCD a contiguous range of tiles so that neighbouring tiles, whose
// output runs for a bucket are adjacent, share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t G)
{
    const uint32_t q = G >> 3, r = G & 7u, x = b & 7u, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ uint32_t find_by_tile(const Seg* segs, uint32_t nsegs, uint32_t t)
{
    uint32_t lo = 0, hi = nsegs - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (segs[mid].tile0 <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ uint32_t find_by_chunk(const Seg* segs, uint32_t nsegs, uint32_t c)
{
    uint32_t lo = 0, hi = nsegs - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (segs[mid].chunk0 <= c) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__host__ __device__ __forceinline__ uint32_t ceil_log2_u32(uint32_t x)
{
    uint32_t r = 0;
    while ((1ull << r) < (uint64_t)x) ++r;
    return r;
}

// Light bucket bits for a subproblem of `len` records so that buckets hold
// about alpha/4 records, leaving room below alpha for the spread of bucket
// sizes (at least 1 bit, at most kLightBitsMax and the hash bits left).
__host__ __device__ __forceinline__ uint32_t choose_nl(uint32_t len, uint32_t alpha, uint32_t cap,
                                                       uint32_t shift, uint32_t hash_bits = 64)
{
    uint32_t target = alpha / 4 ? alpha / 4 : 1;
    uint32_t q = (len + target - 1) / target;
    uint32_t nl = ceil_log2_u32(q);
    if (nl < 1) nl = 1;
    if (nl > cap) nl = cap;
    if (nl > hash_bits - shift) nl = hash_bits - shift;
    return nl;
}

// Subarray size for a level of `total` records: about 2048 subarrays,
// a power of two within [tmin, tmax].
__host__ __device__ __forceinline__ uint32_t choose_tile(uint64_t total, uint32_t tmin, uint32_t tmax)
{
    uint64_t want = total / 2048;
    uint32_t t = tmin;
    while ((uint64_t)t * 2 <= want && t * 2 <= tmax) t *= 2;
    return t;
}

// ================================================================ Step 1
// Sampling and Bucketing (Section 3.1): |S| = ceil(c ln n') sampled keys,
// sorted by hash in LDS; keys seen at least tau times are heavy and get ids
// n_L, n_L + 1, ... in ascending hash order; a two-choice heavy table is
// built for the later passes.  One block per subproblem.

// Compare-exchange of a bitonic stage: ascending where (index & k) == 0.
__device__ __forceinline__ void bitonic_cx(uint64_t& x, uint64_t& y, bool up)
{
    const bool sw = (x > y) == up;
    const uint64_t a = sw ? y : x, b = sw ? x : y;
    x = a;
    y = b;
}

// Stages of one k whose distance j is below C, on the thread's C contiguous
// elements held in registers; base = logical index of e[0].
template <int C>
__device__ __forceinline__ void bitonic_regs(uint64_t (&e)[C], uint32_t base, uint32_t k, uint32_t jmax)
{
#pragma unroll
    for (int j = C / 2; j >= 1; j >>= 1) {
        if ((uint32_t)j > jmax) continue;
#pragma unroll
        for (int q = 0; q < C; ++q)
            if ((q & j) == 0) bitonic_cx(e[q], e[q + j], ((base + q) & k) == 0);
    }
}

// The sample, gathered straight into registers: thread t holds samples
// t*C .. t*C + C - 1 (h(key) when hashed, else the key); positions past s are
// padded with ~0.  Positions are drawn with replacement from the
// counter-based generator; all loads of a thread are issued before use.
// Stream key of the sample positions of a subproblem at a level.
__device__ __forceinline__ uint64_t sample_stream(const LevelArgs& a, const Seg& sg)
{
    const uint64_t golden = 0x9e3779b97f4a7c15ULL;
    const uint64_t k0 = splitmix_mix(a.seed + golden * ((uint64_t)a.level + 1));
    return splitmix_mix(k0 ^ (uint64_t)(sg.start - sg.ibase));
}

// Position of sample i (drawn with replacement) in the subproblem's records.
__device__ __forceinline__ uint64_t sample_pos(uint64_t k1, const Seg& sg, uint32_t i)
{
    const uint64_t x = splitmix_mix(k1 + 0x9e3779b97f4a7c15ULL * ((uint64_t)i + 1));
    return (uint64_t)sg.start + __umul64hi(x, (uint64_t)sg.len);
}

template <int MODE, int C, typename K>
__device__ __forceinline__ void gather_regs(const LevelArgs& a, const Seg& sg, uint32_t s, bool hashed,
                                            uint64_t (&e)[C])
{
    const uint64_t k1 = sample_stream(a, sg);
    const uint32_t base = threadIdx.x * C;
    if constexpr (kWide<K>) {
        // 128-bit keys: always hashed; the level hash of each sampled key
        Key128 kv[C];
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const uint32_t i = base + q;
            if (i < s) kv[q] = ((const K*)a.src_keys)[sample_pos(k1, sg, i)];
        }
#pragma unroll
        for (int q = 0; q < C; ++q)
            e[q] = base + q < s ? level_hash(khash<MODE>(kv[q]), sg.shift) : ~0ull;
    } else {
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const uint32_t i = base + q;
            e[q] = ~0ull;
            if (i < s) e[q] = (uint64_t)((const K*)a.src_keys)[sample_pos(k1, sg, i)];
        }
        if (hashed) {
#pragma unroll
            for (int q = 0; q < C; ++q)
                if (base + q < s) e[q] = user_hash<MODE>(e[q]);
        }
    }
}

// Ascending bitonic sort of P = C * nt elements, thread t < nt holding the
// logical elements t*C + q in e[q] (nt = BS for C >= 2; nt = P <= BS for
// C = 1).  Stages of distance j < C run in registers.  Distances from C up to
// 64*C pair element t*C + q with element (t ^ j/C)*C + q, held by another lane
// of the same wave in the same register: those stages exchange registers
// across lanes, with no LDS round trip and no block barrier.  Longer stages go
// through LDS in a q-major layout (element t*C + q at smp[q*nt + t]) with
// pairs handed out so that neighbouring lanes touch neighbouring words.  On
// return e[] is sorted in the same layout and smp holds the sorted sequence
// in logical order.
template <int BS, int C>
__device__ void bitonic_sort_block(uint64_t (&e)[C], uint64_t* smp, uint32_t P)
{
    const uint32_t t = threadIdx.x;
    const uint32_t nt = P / C;
    const bool own = t < nt;
    const uint32_t base = t * C;
    constexpr uint32_t kWaveSpan = 64u * (uint32_t)C;  // elements of one wave
#pragma unroll
    for (uint32_t k = 2; k <= (uint32_t)C; k <<= 1) bitonic_regs<C>(e, base, k, k >> 1);
    for (uint32_t k = 2 * C; k <= P; k <<= 1) {
        uint32_t j = k >> 1;
        if (j >= kWaveSpan) {
            if (own) {
#pragma unroll
                for (int q = 0; q < C; ++q) smp[q * nt + t] = e[q];
            }
            __syncthreads();
            for (; j >= kWaveSpan; j >>= 1) {
                const uint32_t jt = j / C;  // distance in threads
                for (uint32_t pp = t; pp < (P >> 1); pp += BS) {
                    const uint32_t q = pp / (nt >> 1);
                    const uint32_t u = pp % (nt >> 1);
                    const uint32_t ta = ((u & ~(jt - 1)) << 1) | (u & (jt - 1));
                    uint64_t* pa = smp + q * nt + ta;
                    uint64_t x = pa[0], y = pa[jt];
                    bitonic_cx(x, y, ((ta * C + q) & k) == 0);
                    pa[0] = x;
                    pa[jt] = y;
                }
                __syncthreads();
            }
            if (own) {
#pragma unroll
                for (int q = 0; q < C; ++q) e[q] = smp[q * nt + t];
            }
            __syncthreads();
        }
        // the lower element of a pair keeps the minimum in an ascending run
        const bool up = (base & k) == 0;
        for (; j >= (uint32_t)C; j >>= 1) {
            const uint32_t d = j / C;  // lane distance, below 64
            const bool keep_min = ((t & d) == 0) == up;
#pragma unroll
            for (int q = 0; q < C; ++q) {
                const uint64_t y = __shfl_xor(e[q], (int)d, 64);
                const uint64_t x = e[q];
                e[q] = keep_min ? (y < x ? y : x) : (y < x ? x : y);
            }
        }
        bitonic_regs<C>(e, base, k, C / 2);
    }
    if (own) {
#pragma unroll
        for (int q = 0; q < C; ++q) smp[base + q] = e[q];
    }
    __syncthreads();
}

// Heavy keys of the sorted sample (thread t holds sorted elements t*C + q in
// e[q], smp the whole sequence in order).  Run lengths of the distinct hashes
// (histogram of min(length, 63)); the heavy table holds kHeavyMax keys, so if
// more runs reach tau, the threshold rises to the least value that leaves at
// most kHeavyMax of them (the most frequent keys stay heavy; at most
// 16384/32 = 512 runs can reach 32, so the search ends below 63).  Heavy
// hashes go to hv and heavy_list in ascending order; returns n_H and adds the
// samples on heavy keys to *sh_hs.
template <int BS, int C>
__device__ uint32_t select_heavy_runs(const uint64_t (&e)[C], const uint64_t* smp, uint32_t s, uint32_t tau,
                                      uint32_t* rh, uint32_t* tmp, uint32_t* sh_te, uint32_t* sh_hs, uint64_t* hv,
                                      uint64_t* heavy_out, unsigned long long* top2)
{
    const uint32_t t = threadIdx.x;
    const uint32_t base = t * C;
    uint32_t rl[C];
    uint64_t prev = (base > 0 && base - 1 < s) ? smp[base - 1] : 0ull;
#pragma unroll
    for (int q = 0; q < C; ++q) {
        const uint32_t i = base + q;
        rl[q] = 0;
        const uint64_t pv = q ? e[q - 1] : prev;
        if (i < s && (i == 0 || e[q] != pv)) {
            // run end: within the thread's registers if it ends there, else a
            // binary search over smp for the first position in (i, s] past it
            uint32_t len = 1;
            bool open = true;
#pragma unroll
            for (int r = q + 1; r < C; ++r) {
                if (open && base + r < s && e[r] == e[q]) ++len;
                else open = false;
            }
            if (open && base + C < s && smp[base + C] == e[q]) {
                uint32_t l = base + C, r = s;
                while (r - l > 1) {
                    const uint32_t mid = (l + r) >> 1;
                    if (smp[mid] == e[q]) l = mid;
                    else r = mid;
                }
                len = r - i;
            } else if (open && base + C >= s) {
                len = s - i;
            }
            rl[q] = len;
            atomicAdd(&rh[len < 63 ? len : 63], 1u);
        }
    }
    __syncthreads();
    if (t == 0) {
        uint32_t tt = tau < 1 ? 1u : tau;
        while (tt < 63) {
            uint32_t c = 0;
            for (uint32_t L = tt; L < 64; ++L) c += rh[L];
            if (c <= kHeavyMax) break;
            ++tt;
        }
        *sh_te = tt;
    }
    __syncthreads();
    const uint32_t te = *sh_te;
    uint32_t cnt = 0, hs = 0;
#pragma unroll
    for (int q = 0; q < C; ++q)
        if (rl[q] >= te) {
            ++cnt;
            hs += rl[q];
        }
    uint32_t total = 0;
    uint32_t id = block_excl_scan<BS>(cnt, tmp, &total);
#pragma unroll
    for (int q = 0; q < C; ++q)
        if (rl[q] >= te) {
            if (id < kHeavyMax) {
                hv[id] = e[q];
                heavy_out[id] = e[q];
                // the two most sampled heavy keys: (run length, id) maxima
                const unsigned long long tag = ((unsigned long long)rl[q] << 16) | id;
                const unsigned long long prev = atomicMax(&top2[0], tag);
                atomicMax(&top2[1], prev < tag ? prev : tag);
            }
            ++id;
        }
    if (hs) atomicAdd(sh_hs, hs);
    __syncthreads();
    return total < kHeavyMax ? total : kHeavyMax;
}

// Gather, sort and heavy selection for one sample size class (P = C * BS,
// or P <= BS with C = 1).  Returns n_H.
template <int MODE, int BS, int C, typename K>
__device__ uint32_t sample_select(const LevelArgs& a, const Seg& sg, uint32_t sid, uint32_t s, uint32_t tau,
                                  uint32_t P, uint64_t* smp, uint32_t* rh, uint32_t* tmp, uint32_t* sh_te,
                                  uint32_t* sh_hs, uint64_t* hv, unsigned long long* top2)
{
    uint64_t e[C];
    gather_regs<MODE, C, K>(a, sg, s, true, e);
    bitonic_sort_block<BS, C>(e, smp, P);
    return select_heavy_runs<BS, C>(e, smp, s, tau, rh, tmp, sh_te, sh_hs, hv,
                                    a.heavy_list + (size_t)sid * kHeavyMax, top2);
}

// Gather and sort of raw keys (semisort_<): smp holds the sorted sample.
template <int BS, int C, typename K>
__device__ void sample_sort_keys(const LevelArgs& a, const Seg& sg, uint32_t s, uint32_t P, uint64_t* smp)
{
    uint64_t e[C];
    gather_regs<0, C, K>(a, sg, s, false, e);
    bitonic_sort_block<BS, C>(e, smp, P);
}

template <int MODE, typename K>
__device__ __forceinline__ void sample_heavy_item(const LevelArgs& a, uint32_t sid)
{
    constexpr int BS = 1024;
    __shared__ uint64_t smp[kSampleMax];
    __shared__ uint64_t hv[kHeavyMax];
    __shared__ uint32_t owner[2 * kHeavySlotsMax];
    __shared__ uint32_t tmp[20];
    __shared__ uint32_t rh[64];
    __shared__ uint32_t sh_s, sh_tau, sh_te, sh_hs, sh_nl, sh_fail;
    __shared__ unsigned long long sh_top[2];

    const uint32_t tid = threadIdx.x;
    const Seg sg = a.segs[sid];
    if (tid < 2) sh_top[tid] = 0;
    if (tid == 0) {
        // |S| = ceil(c ln n'), at most n'/8 (small subproblems are not
        // sampled almost entirely) and at most the LDS capacity
        const double L = log((double)sg.len);
        const double cm = a.level ? (double)a.sample_mult / (double)a.deep_div : (double)a.sample_mult;
        double sd = ceil(cm * L);
        uint32_t s = sg.len < 2 ? 0u : (uint32_t)sd;
        if (s > sg.len / 8) s = sg.len / 8;
        if (s > kSampleMax) s = kSampleMax;
        sh_s = s;
        sh_tau = a.heavy_min ? a.heavy_min : (sg.len < 3 ? 1u : (uint32_t)ceil(L));
        sh_hs = 0;
    }
    if (tid < 64) rh[tid] = 0;
    __syncthreads();
    const uint32_t s = sh_s, tau = sh_tau;
    uint32_t P = 2;
    while (P < s) P <<= 1;
    uint32_t nh;
    if (P == 16 * BS) nh = sample_select<MODE, BS, 16, K>(a, sg, sid, s, tau, P, smp, rh, tmp, &sh_te, &sh_hs, hv, sh_top);
    else if (P == 8 * BS) nh = sample_select<MODE, BS, 8, K>(a, sg, sid, s, tau, P, smp, rh, tmp, &sh_te, &sh_hs, hv, sh_top);
    else if (P == 4 * BS) nh = sample_select<MODE, BS, 4, K>(a, sg, sid, s, tau, P, smp, rh, tmp, &sh_te, &sh_hs, hv, sh_top);
    else if (P == 2 * BS) nh = sample_select<MODE, BS, 2, K>(a, sg, sid, s, tau, P, smp, rh, tmp, &sh_te, &sh_hs, hv, sh_top);
    else nh = sample_select<MODE, BS, 1, K>(a, sg, sid, s, tau, P, smp, rh, tmp, &sh_te, &sh_hs, hv, sh_top);

    // Light bucket count.  With adaptive_nl, n_L is the smallest power of two
    // that lets the light records finish in the fewest levels: one level if
    // buckets of ~alpha/2 can be reached with at most nl_bits bits, else two.
    if (tid == 0) {
        uint32_t nl = sg.nl_bits;
        if (a.adaptive_nl && s) {
            const double light = (double)sg.len * (double)(s - sh_hs) / (double)s;
            const double target = (double)a.alpha * (double)a.nl_target / 100.0;
            const uint32_t cap = sg.nl_bits;
            uint32_t nl1 = 1;
            while (nl1 < 31 && (double)(1u << nl1) * target < light) ++nl1;
            if (nl1 <= cap) {
                nl = nl1;
            } else {
                uint32_t nl2 = 1;
                while (nl2 < 31 && (double)(1u << nl2) * (double)(1u << kLightBitsMax) * target < light) ++nl2;
                if (nl2 <= cap) nl = nl2;
            }
        }
        sh_nl = nl;
    }

    // Two-choice (cuckoo) heavy table: two tables of 2^hlog2 slots, at most a
    // quarter full.  Built in parallel: each key is placed by atomic exchange
    // and an evicted key moves on to its slot in the other table.  If some
    // chain grows too long, the salt of the second hash changes and the build
    // starts again.  The layout may vary from run to run; every key sits in
    // one of its two slots, so lookups do not.
    uint32_t hlog2 = 0;
    if (nh) {
        hlog2 = ceil_log2_u32(2 * nh);
        if (hlog2 < 4) hlog2 = 4;
    }
    const uint32_t direct = (MODE == 0 && !kWide<K> && sg.shift < 32) ? kDirectSlots : 0u;
    const uint32_t slots = nh ? (1u << hlog2) : 0u;
    uint32_t salt = 0;
    bool built = nh == 0;
    while (!built) {
        for (uint32_t i = tid; i < 2 * kHeavySlotsMax; i += BS) owner[i] = kEmpty32;
        if (tid == 0) sh_fail = 0;
        __syncthreads();
        if (tid < nh) {
            uint32_t cur = tid;
            int side = 0;
            for (uint32_t it = 0;; ++it) {
                if (it >= 64) {
                    atomicOr(&sh_fail, 1u);
                    break;
                }
                const uint64_t h = hv[cur];
                const uint32_t hf = hlog2 | (salt << 8) | direct;
                const uint32_t sl = side == 0 ? heavy_slot(h, hf, 0) : kHeavySlotsMax + heavy_slot(h, hf, 1);
                const uint32_t prev = atomicExch(&owner[sl], cur);
                if (prev == kEmpty32) break;
                cur = prev;  // the evicted key moves to its other table
                side = (sl < kHeavySlotsMax) ? 1 : 0;
            }
        }
        __syncthreads();
        built = sh_fail == 0;
        if (built || salt == 15) break;
        ++salt;
        __syncthreads();
    }
    __syncthreads();
    if (!built && tid == 0) atomicOr(&a.info->status, kStatusHeavyTable);
    const uint32_t hfield = nh ? (hlog2 | (salt << 8) | direct) : 0u;
    const uint32_t nL = 1u << sh_nl;
    for (uint32_t i = tid; i < 2 * kHeavySlotsMax; i += BS) {
        const bool used = (i & (kHeavySlotsMax - 1)) < slots;
        if (!used) continue;
        const uint32_t o = owner[i];
        a.tab_h[(size_t)sid * 2 * kHeavySlotsMax + i] = o != kEmpty32 ? hv[o] : 0ull;
        a.tab_id[(size_t)sid * 2 * kHeavySlotsMax + i] = o != kEmpty32 ? (uint16_t)(nL + o) : kEmpty16;
    }
    for (uint32_t b = tid; b < nL + nh; b += BS) a.bfin[(size_t)sid * kNbStride + b] = b >= nL ? 1 : 0;
    if constexpr (kWide<K>) {
        // One sampled key per heavy id: the lowest-numbered sample whose level
        // hash is the id's.  The counting pass sends a record to the heavy
        // bucket only if its key equals this one, so the bucket holds one key
        // whatever collides with its hash.  Every heavy hash came from the
        // sample, so each id finds a key; were one missing, its records would
        // all stay light, which is still correct.
        uint32_t* repi = (uint32_t*)smp;  // the sample is no longer needed
        for (uint32_t h = tid; h < nh; h += BS) repi[h] = kEmpty32;
        __syncthreads();
        const uint64_t k1 = sample_stream(a, sg);
        const K* src = (const K*)a.src_keys;
        if (nh && built) {
            for (uint32_t i = tid; i < s; i += BS) {
                const uint64_t h = level_hash(khash<MODE>(src[sample_pos(k1, sg, i)]), sg.shift);
                const uint32_t o1 = owner[heavy_slot(h, hfield, 0)];
                const uint32_t o2 = owner[kHeavySlotsMax + heavy_slot(h, hfield, 1)];
                const uint32_t o = (o1 != kEmpty32 && hv[o1] == h) ? o1 : (o2 != kEmpty32 && hv[o2] == h) ? o2 : kEmpty32;
                if (o != kEmpty32) atomicMin(&repi[o], i);
            }
        }
        __syncthreads();
        for (uint32_t h = tid; h < nh; h += BS) {
            const uint32_t i = repi[h];
            Key128 k{~0ull, ~0ull};
            if (i != kEmpty32) k = src[sample_pos(k1, sg, i)];
            ((Key128*)a.hrep)[(size_t)sid * kHeavyMax + h] = k;
        }
    } else {
        for (uint32_t h = tid; h < nh; h += BS) a.bkey[(size_t)sid * kNbStride + nL + h] = key_of_hash<MODE>(hv[h]);
    }
    if (a.reduce)
        for (uint32_t h = tid; h < nh; h += BS) a.hsum[(size_t)sid * kHeavyMax + h] = red_identity(a.rop);
    if (tid == 0) {
        // heavy ids of the two most sampled keys, for the counting pass
        const uint32_t t0 = sh_top[0] ? nL + (uint32_t)(sh_top[0] & 0xFFFFu) : 0xFFFFu;
        const uint32_t t1 = sh_top[1] ? nL + (uint32_t)(sh_top[1] & 0xFFFFu) : 0xFFFFu;
        a.top[sid] = t0 | (t1 << 16);
        a.segs[sid].nheavy = (uint16_t)nh;
        a.segs[sid].hlog2 = (uint16_t)hfield;
        a.segs[sid].nl_bits = (uint8_t)sh_nl;
        a.segs[sid].nbk = (uint16_t)(nL + nh);
        if (sid == 0) {
            a.info->smp_total = s;
            a.info->smp_heavy = sh_hs;
        }
    }
}

template <int MODE, typename K = uint64_t>
__global__ __launch_bounds__(1024) void k_sample_heavy(LevelArgs a)
{
    sample_heavy_item<MODE, K>(a, blockIdx.x);
}

// Device-sized levels: a resident grid walks the subproblems counted in dims.
__device__ __forceinline__ uint32_t ds_nsegs(const LevelArgs& a)
{
    const uint32_t n = a.dims->nsegs;
    return n < a.seg_cap ? n : a.seg_cap;
}

template <int MODE>
__global__ __launch_bounds__(1024) void k_sample_heavy_ds(LevelArgs a)
{
    const uint32_t n = ds_nsegs(a);
    for (uint32_t sid = blockIdx.x; sid < n; sid += gridDim.x) {
        sample_heavy_item<MODE, uint64_t>(a, sid);
        __syncthreads();
    }
}

// ================================================================ Step 2a
// Counting pass (Section 3.2): per subarray, sequential over its records in
// the paper; here one block per subarray with LDS counters.  Counting is
// order-free, so plain LDS atomics suffice.

template <int MODE, typename K>
__device__ __forceinline__ void count_item(const LevelArgs& a, uint32_t t, uint32_t nsegs, uint32_t tile)
{
    constexpr int BS = 1024;
    __shared__ uint32_t cnt[kNbStride];
    __shared__ uint8_t finl[kNbStride];
    __shared__ uint64_t th[2 * kHeavySlotsMax];
    __shared__ uint16_t tidh[2 * kHeavySlotsMax];
    __shared__ Key128 rep[kWide<K> ? kHeavyMax : 1];  // 128-bit keys: the sampled key of each heavy id

    const uint32_t tid = threadIdx.x;
    const uint32_t sid = find_by_tile(a.segs, nsegs, t);
    const Seg sg = a.segs[sid];
    const uint32_t lt = t - sg.tile0;
    const uint64_t r0 = (uint64_t)sg.start + (uint64_t)lt * tile;
    const uint64_t send = (uint64_t)sg.start + sg.len;
    const uint64_t r1 = r0 + tile < send ? r0 + tile : send;
    const uint32_t nL = 1u << sg.nl_bits;
    const uint32_t nb = sg.nbk;
    const uint32_t hlog2 = sg.hlog2;  // slot bits and salt
    const uint32_t slots = (hlog2 & 0xFFu) ? (1u << (hlog2 & 0xFFu)) : 0u;

    for (uint32_t b = tid; b < nb; b += BS) {
        cnt[b] = 0;
        finl[b] = a.reduce ? a.bfin[(size_t)sid * kNbStride + b] : 0;
    }
    for (uint32_t i = tid; i < 2 * slots; i += BS) {
        const uint32_t j = i < slots ? i : kHeavySlotsMax + (i - slots);
        th[j] = a.tab_h[(size_t)sid * 2 * kHeavySlotsMax + j];
        tidh[j] = a.tab_id[(size_t)sid * 2 * kHeavySlotsMax + j];
    }
    if constexpr (kWide<K>) {
        const uint32_t nh = nb - nL < kHeavyMax ? nb - nL : kHeavyMax;
        for (uint32_t h = tid; h < nh; h += BS) rep[h] = ((const Key128*)a.hrep)[(size_t)sid * kHeavyMax + h];
    }
    __syncthreads();

    const uint32_t shift = sg.shift;
    const uint32_t lmask = nL - 1;
    const K* keys = (const K*)a.src_keys;
    uint16_t* bids = a.bids;
    // The two most frequent heavy buckets are counted per wave by ballot
    // (one LDS update per wave instead of one per record); the others by
    // LDS atomics.  Collect-reduce does not count heavy records at all.
    const uint32_t tp = a.reduce ? 0xFFFFFFFFu : a.top[sid];
    const uint32_t top0 = tp & 0xFFFFu, top1 = tp >> 16;
    const uint32_t lane = tid & 63u;
    auto tally = [&](uint32_t b) {
        const uint64_t b0 = __ballot(b == top0), b1 = __ballot(b == top1);
        if (b == top0) {
            if (lane == (uint32_t)__ffsll((long long)b0) - 1) atomicAdd(&cnt[top0], (uint32_t)__popcll(b0));
        } else if (b == top1) {
            if (lane == (uint32_t)__ffsll((long long)b1) - 1) atomicAdd(&cnt[top1], (uint32_t)__popcll(b1));
        } else if (!finl[b]) {
            atomicAdd(&cnt[b], 1u);
        }
    };
    constexpr int U = 8;  // loads in flight per thread
    // 32-bit offsets from the subarray's start (uniform base pointers)
    const K* kt = keys + r0;
    uint16_t* bt = bids + r0;
    const uint32_t len = (uint32_t)(r1 - r0);
    // GetBucketId of one key.  128-bit keys: a heavy id holds only its
    // sampled key; another key with the same level hash takes its light bucket.
    auto bucket_key = [&](const KReg<K>& k, auto kind) -> uint32_t {
        constexpr int TK = decltype(kind)::value;  // heavy table kind
        if constexpr (kWide<K>) {
            const Hash2 hh = khash<MODE>(k);
            const uint64_t w = hash_window(hh, shift);
            const uint32_t b = bucket_of_w<TK>(level_hash(hh, shift), w, th, tidh, hlog2, lmask);
            return (b >= nL && !(k == rep[b - nL])) ? ((uint32_t)w & lmask) : b;
        } else {
            return bucket_of<TK>(user_hash<MODE>(k), th, tidh, hlog2, shift, lmask);
        }
    };
    auto pass = [&](auto kind) {
        uint32_t o = tid;
        for (; o + (U - 1) * BS < len; o += U * BS) {
            KReg<K> kk[U];
#pragma unroll
            for (int u = 0; u < U; ++u) kk[u] = kload(kt + o + u * BS);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t b = bucket_key(kk[u], kind);
                bt[o + u * BS] = (uint16_t)b;
                tally(b);
            }
        }
        for (; o < len; o += BS) {
            const uint32_t b = bucket_key(kload(kt + o), kind);
            bt[o] = (uint16_t)b;
            tally(b);
        }
    };
    if (!(hlog2 & 0xFFu)) pass(std::integral_constant<int, 0>{});
    else if (hlog2 & kDirectSlots) pass(std::integral_constant<int, 1>{});
    else pass(std::integral_constant<int, 2>{});
    __syncthreads();
    // collect-reduce: heavy records stay where they are; each heavy bucket
    // keeps one slot (in the subproblem's first subarray) for its result
    uint32_t* row = a.C + (size_t)t * kNbStride;
    for (uint32_t b = tid; b < nb; b += BS) row[b] = cnt[b] + ((finl[b] && lt == 0) ? 1u : 0u);
}

template <int MODE, typename K = uint64_t>
__global__ __launch_bounds__(1024) void k_count(LevelArgs a)
{
    count_item<MODE, K>(a, xcd_remap(blockIdx.x, gridDim.x), a.nsegs, a.tile);
}

// Work queue of a resident grid: the n items are split into eight contiguous
// ranges, one per XCD (block b runs on XCD b mod 8 when the grid is first
// dispatched), and the blocks of an XCD take the items of its range in order
// from a counter.  Neighbouring items then run at the same time on one XCD
// and share its L2, as with one block per item.  Every range has blocks
// (the grid is a multiple of 8), so every item is taken whatever the
// placement.  Returns the next item, or n when the block's range is done.
__device__ __forceinline__ uint32_t xcd_queue_next(uint32_t* ctr8, uint32_t n, uint32_t* sh)
{
    const uint32_t x = blockIdx.x & 7u;
    const uint32_t lo = (uint32_t)((uint64_t)n * x / 8), hi = (uint32_t)((uint64_t)n * (x + 1) / 8);
    __syncthreads();  // the previous item's readers of *sh are done
    if (threadIdx.x == 0) *sh = lo + atomicAdd(ctr8 + x, 1u);
    __syncthreads();
    const uint32_t t = *sh;
    return t < hi ? t : n;
}

template <int MODE>
__global__ __launch_bounds__(1024) void k_count_ds(LevelArgs a)
{
    __shared__ uint32_t sh_t;
    const uint32_t ns = ds_nsegs(a), n = a.dims->tiles, tile = a.dims->tile;
    for (uint32_t t = xcd_queue_next(a.q, n, &sh_t); t < n; t = xcd_queue_next(a.q, n, &sh_t))
        count_item<MODE, uint64_t>(a, t, ns, tile);
}

// ================================================================ semisort_<
// Order-preserving buckets (semisort_< with groups in ascending key order).
// The sample is sorted by key; keys sampled at least ceil(ln n') times are
// heavy and get equality buckets; splitters are taken evenly from the
// remaining sorted samples.  Boundaries B_0 < ... < B_{m-1} (splitters and
// heavy keys) give buckets in key order: range R_0, then for each boundary
// its equality bucket (heavy keys only) and the next range.  A key k falls
// in R_j with j = #{boundaries <= k}, unless B_{j-1} = k is heavy.  Per
// subproblem the boundaries go to tab_h and, in tab_id, rid[j] = id of R_j
// (bit 15 of rid[j], j < m: B_j is heavy; its equality bucket is rid[j] + 1).

__device__ __forceinline__ uint32_t lower_bound_u64(const uint64_t* a, uint32_t n, uint64_t x)
{
    uint32_t lo = 0, len = n;
    while (len > 0) {
        const uint32_t half = len >> 1;
        if (a[lo + half] < x) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

__device__ __forceinline__ uint32_t upper_bound_u64(const uint64_t* a, uint32_t n, uint64_t x)
{
    uint32_t lo = 0, len = n;
    while (len > 0) {
        const uint32_t half = len >> 1;
        if (a[lo + half] <= x) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

// Lookup table for the boundary search of the counting pass.  A key's offset
// x = k - B_0 from the smallest boundary falls in a cell: x itself below 64,
// else 64 cells per octave (the octave of x and its next six bits), so the
// cells are monotone in x and about as fine where boundaries are dense
// (skewed keys) as where they are sparse.  lut[c] = number of boundaries in
// cells below c; a key of cell c then has its upper bound among the
// boundaries lut[c] .. lut[c + 1] - 1, usually a handful.
constexpr uint32_t kLessCells = 64 + 58 * 64;  // octaves 6 .. 63

__device__ __forceinline__ uint32_t less_cell(uint64_t x)
{
    if (x < 64) return (uint32_t)x;
    const uint32_t e = 63u - (uint32_t)__clzll((long long)x);  // 6 .. 63
    return 64u + (e - 6u) * 64u + (uint32_t)(x >> (e - 6u)) - 64u;
}

// Smallest offset whose cell is c (c < kLessCells).
__device__ __forceinline__ uint64_t less_cell_start(uint32_t c)
{
    if (c < 64) return c;
    const uint32_t e = (c - 64u) / 64u + 6u, m = (c - 64u) % 64u;
    return (uint64_t)(64u + m) << (e - 6u);
}

// Bucket of k: j = #{boundaries <= k} (upper bound), searched only inside
// k's cell; the equality bucket when B_{j-1} = k is heavy, else R_j.
__device__ __forceinline__ uint32_t less_bucket_lut(uint64_t k, const uint64_t* bnd, const uint16_t* rid,
                                                    const uint16_t* lut, uint32_t m)
{
    uint32_t j = 0;
    if (m != 0 && k >= bnd[0]) {
        const uint32_t c = less_cell(k - bnd[0]);
        const uint32_t a0 = lut[c], a1 = lut[c + 1];
        j = a0 + upper_bound_u64(bnd + a0, a1 - a0, k);
    }
    if (j > 0 && (rid[j - 1] & 0x8000u) && bnd[j - 1] == k) return (rid[j - 1] & 0x7FFFu) + 1;
    return rid[j] & 0x7FFFu;
}

template <typename K = uint64_t>
__global__ __launch_bounds__(1024) void k_sample_less(LevelArgs a)
{
    constexpr int BS = 1024;
    __shared__ uint64_t smp[kSampleMax];
    __shared__ uint64_t spl[kNbStride];
    __shared__ uint64_t hv[kHeavyMax];
    __shared__ uint32_t hf[kNbStride];
    __shared__ uint32_t tmp[20];
    __shared__ uint32_t sh_s, sh_tau, sh_R, sh_nl;

    const uint32_t sid = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const Seg sg = a.segs[sid];
    if (tid == 0) {
        const double L = log((double)sg.len);
        const double cm = a.level ? (double)a.sample_mult / (double)a.deep_div : (double)a.sample_mult;
        double sd = ceil(cm * L);
        uint32_t s = sg.len < 2 ? 0u : (uint32_t)sd;
        if (s > sg.len / 8) s = sg.len / 8;
        if (s > kSampleMax) s = kSampleMax;
        sh_s = s;
        sh_tau = a.heavy_min ? a.heavy_min : (sg.len < 3 ? 1u : (uint32_t)ceil(L));
    }
    __syncthreads();
    const uint32_t s = sh_s, tau = sh_tau;
    uint32_t P = 2;
    while (P < s) P <<= 1;
    if (P == 16 * BS) sample_sort_keys<BS, 16, K>(a, sg, s, P, smp);
    else if (P == 8 * BS) sample_sort_keys<BS, 8, K>(a, sg, s, P, smp);
    else if (P == 4 * BS) sample_sort_keys<BS, 4, K>(a, sg, s, P, smp);
    else if (P == 2 * BS) sample_sort_keys<BS, 2, K>(a, sg, s, P, smp);
    else sample_sort_keys<BS, 1, K>(a, sg, s, P, smp);
    // heavy keys in ascending key order; per sample: heavy or not, and the
    // rank of the non-heavy ones
    const uint32_t per = (s + BS - 1) / BS;
    const uint32_t lo = tid * per;
    const uint32_t hi = lo + per < s ? lo + per : s;
    // threshold raised, if needed, so that at most kHeavyMax keys are heavy
    // (the same rule as for semisort_=)
    __shared__ uint32_t rh[64];
    __shared__ uint32_t sh_te;
    if (tid < 64) rh[tid] = 0;
    __syncthreads();
    for (uint32_t i = lo; i < hi; ++i) {
        if (i != 0 && smp[i] == smp[i - 1]) continue;
        const uint32_t len = upper_bound_u64(smp, s, smp[i]) - i;
        atomicAdd(&rh[len < 63 ? len : 63], 1u);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t t = tau < 1 ? 1u : tau;
        while (t < 63) {
            uint32_t c = 0;
            for (uint32_t L = t; L < 64; ++L) c += rh[L];
            if (c <= kHeavyMax) break;
            ++t;
        }
        sh_te = t;
    }
    __syncthreads();
    const uint32_t te = sh_te;
    uint32_t nhs = 0, nls = 0;
    for (uint32_t i = lo; i < hi; ++i) {
        const bool start = (i == 0) || smp[i] != smp[i - 1];
        if (start && i + te - 1 < s && smp[i + te - 1] == smp[i]) ++nhs;
        const uint32_t lb = lower_bound_u64(smp, s, smp[i]);
        const uint32_t ub = upper_bound_u64(smp, s, smp[i]);
        if (ub - lb < te) ++nls;
    }
    uint32_t tot_h = 0, tot_l = 0;
    uint32_t hid = block_excl_scan<BS>(nhs, tmp, &tot_h);
    uint32_t lrank = block_excl_scan<BS>(nls, tmp, &tot_l);
    const uint32_t nh = tot_h < kHeavyMax ? tot_h : kHeavyMax;
    if (tot_h > kHeavyMax && tid == 0) atomicOr(&a.info->status, kStatusHeavyTable);
    if (tid == 0) {
        // number of ranges: the fewest-levels rule on the estimated light
        // records, within the bucket budget and the distinct light samples
        uint32_t nl = sg.nl_bits;
        if (a.adaptive_nl && s) {
            const double light = (double)sg.len * (double)tot_l / (double)s;
            const double target = (double)a.alpha * (double)a.nl_target / 100.0;
            const uint32_t cap = sg.nl_bits;
            uint32_t nl1 = 1;
            while (nl1 < 31 && (double)(1u << nl1) * target < light) ++nl1;
            if (nl1 <= cap) {
                nl = nl1;
            } else {
                uint32_t nl2 = 1;
                while (nl2 < 31 && (double)(1u << nl2) * (double)(1u << kLightBitsMax) * target < light) ++nl2;
                nl = nl2 <= cap ? nl2 : cap;
            }
        }
        uint32_t R = 1u << nl;
        if (R > kNbStride - 2 * nh) R = kNbStride - 2 * nh;
        if (R > tot_l) R = tot_l ? tot_l : 1u;
        sh_R = R;
        sh_nl = nl;
    }
    __syncthreads();
    const uint32_t R = sh_R;
    for (uint32_t i = lo; i < hi; ++i) {
        const bool start = (i == 0) || smp[i] != smp[i - 1];
        if (start && i + te - 1 < s && smp[i + te - 1] == smp[i]) {
            if (hid < kHeavyMax) {
                hv[hid] = smp[i];
                a.heavy_list[(size_t)sid * kHeavyMax + hid] = smp[i];
            }
            ++hid;
        }
        const uint32_t lb = lower_bound_u64(smp, s, smp[i]);
        const uint32_t ub = upper_bound_u64(smp, s, smp[i]);
        if (ub - lb < te) {
            // splitter j (j < R-1) sits at light rank floor((j+1) * tot_l / R);
            // with R <= tot_l the ranks of different j differ, and the only
            // candidate for rank r is j+1 = ceil(r * R / tot_l)
            const uint64_t r = lrank;
            const uint64_t jp1 = (r * R + tot_l - 1) / tot_l;
            if (jp1 >= 1 && jp1 < R && (jp1 * tot_l) / R == r) spl[jp1 - 1] = smp[i];
            ++lrank;
        }
    }
    __syncthreads();
    // distinct splitters, compacted into smp (the sample is no longer needed)
    const uint32_t nc = R - 1;
    const uint32_t per2 = (nc + BS - 1) / BS;
    const uint32_t c0 = tid * per2;
    const uint32_t c1 = c0 + per2 < nc ? c0 + per2 : nc;
    uint32_t nv = 0;
    for (uint32_t j = c0; j < c1; ++j) nv += (j == 0 || spl[j] != spl[j - 1]) ? 1u : 0u;
    uint32_t ns = 0;
    uint32_t vat = block_excl_scan<BS>(nv, tmp, &ns);
    for (uint32_t j = c0; j < c1; ++j)
        if (j == 0 || spl[j] != spl[j - 1]) smp[vat++] = spl[j];
    __syncthreads();
    // merge splitters and heavy keys into the sorted boundary list
    const uint32_t m = ns + nh;
    uint64_t* bnd = a.tab_h + (size_t)sid * 2 * kHeavySlotsMax;
    uint16_t* rid = a.tab_id + (size_t)sid * 2 * kHeavySlotsMax;
    for (uint32_t j = tid; j < ns; j += BS) {
        const uint32_t pos = j + lower_bound_u64(hv, nh, smp[j]);
        bnd[pos] = smp[j];
        hf[pos] = 0;
    }
    for (uint32_t i = tid; i < nh; i += BS) {
        const uint32_t pos = i + lower_bound_u64(smp, ns, hv[i]);
        bnd[pos] = hv[i];
        hf[pos] = 1;
    }
    __syncthreads();
    // rid[j] = j + #heavy boundaries before j, for j = 0..m
    const uint32_t per3 = (m + 1 + BS - 1) / BS;
    const uint32_t d0 = tid * per3;
    const uint32_t d1 = d0 + per3 < m + 1 ? d0 + per3 : m + 1;
    uint32_t hcount = 0;
    for (uint32_t j = d0; j < d1; ++j) hcount += (j < m) ? hf[j] : 0u;
    uint32_t hbefore = block_excl_scan<BS>(hcount, tmp, nullptr);
    const uint32_t nb = m + 1 + nh;
    uint8_t* fin = a.bfin + (size_t)sid * kNbStride;
    for (uint32_t b = tid; b < nb; b += BS) fin[b] = 0;
    __syncthreads();
    for (uint32_t j = d0; j < d1; ++j) {
        const uint32_t r = j + hbefore;
        const bool heavy = j < m && hf[j];
        rid[j] = (uint16_t)(r | (heavy ? 0x8000u : 0u));
        if (heavy) {
            fin[r + 1] = 1;
            a.bkey[(size_t)sid * kNbStride + r + 1] = bnd[j];
        }
        hbefore += heavy ? 1u : 0u;
    }
    if (tid == 0) {
        a.segs[sid].nheavy = (uint16_t)nh;
        a.segs[sid].nbk = (uint16_t)nb;
        a.segs[sid].nl_bits = (uint8_t)sh_nl;
        a.segs[sid].hlog2 = 0;
    }
}

// Counting pass for splitter buckets: binary search over the boundaries in LDS.
template <typename K = uint64_t>
__global__ __launch_bounds__(1024) void k_count_less(LevelArgs a)
{
    constexpr int BS = 1024;
    __shared__ uint32_t cnt[kNbStride];
    __shared__ uint8_t finl[kNbStride];
    __shared__ uint64_t bnd[kNbStride];
    __shared__ uint16_t rid[kNbStride + 1];
    __shared__ uint16_t lut[kLessCells + 1];
    const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t tid = threadIdx.x;
    const uint32_t sid = find_by_tile(a.segs, a.nsegs, t);
    const Seg sg = a.segs[sid];
    const uint32_t lt = t - sg.tile0;
    const uint64_t r0 = (uint64_t)sg.start + (uint64_t)lt * a.tile;
    const uint64_t send = (uint64_t)sg.start + sg.len;
    const uint64_t r1 = r0 + a.tile < send ? r0 + a.tile : send;
    const uint32_t nb = sg.nbk;
    const uint32_t m = nb - 1 - sg.nheavy;
    for (uint32_t b = tid; b < nb; b += BS) {
        cnt[b] = 0;
        finl[b] = a.reduce ? a.bfin[(size_t)sid * kNbStride + b] : 0;
    }
    for (uint32_t j = tid; j <= m; j += BS) {
        if (j < m) bnd[j] = a.tab_h[(size_t)sid * 2 * kHeavySlotsMax + j];
        rid[j] = a.tab_id[(size_t)sid * 2 * kHeavySlotsMax + j];
    }
    __syncthreads();
    if (m != 0) {
        const uint64_t lo = bnd[0];
        for (uint32_t c = tid; c <= kLessCells; c += BS) {
            // boundaries whose offset lies in a cell below c
            const uint64_t x = c < kLessCells ? less_cell_start(c) : ~0ull;
            lut[c] = (uint16_t)(x > bnd[m - 1] - lo ? m : lower_bound_u64(bnd, m, lo + x));
        }
    }
    __syncthreads();
    constexpr int U = 8;
    const K* kt = (const K*)a.src_keys + r0;
    uint16_t* bt = a.bids + r0;
    const uint32_t len = (uint32_t)(r1 - r0);
    uint32_t o = tid;
    for (; o + (U - 1) * BS < len; o += U * BS) {
        uint64_t kk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) kk[u] = kt[o + u * BS];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t b = less_bucket_lut(kk[u], bnd, rid, lut, m);
            bt[o + u * BS] = (uint16_t)b;
            if (!finl[b]) atomicAdd(&cnt[b], 1u);
        }
    }
    for (; o < len; o += BS) {
        const uint32_t b = less_bucket_lut(kt[o], bnd, rid, lut, m);
        bt[o] = (uint16_t)b;
        if (!finl[b]) atomicAdd(&cnt[b], 1u);
    }
    __syncthreads();
    // collect-reduce: heavy records stay where they are; each heavy bucket
    // keeps one slot (in the subproblem's first subarray) for its result
    uint32_t* row = a.C + (size_t)t * kNbStride;
    for (uint32_t b = tid; b < nb; b += BS) row[b] = cnt[b] + ((finl[b] && lt == 0) ? 1u : 0u);
}

// ================================================================ Step 2b
// Column-major prefix X of the counting matrix (Algorithm 1): per bucket, the
// records of all earlier buckets plus that bucket's records in earlier
// subarrays.  Four passes over the rows: chunk sums, a scan over chunks per
// bucket, bucket starts per subproblem, and the fill of X.

__device__ __forceinline__ void scan_chunks_item(const LevelArgs& a, uint32_t ch, uint32_t nsegs)
{
    const uint32_t sid = find_by_chunk(a.segs, nsegs, ch);
    const Seg sg = a.segs[sid];
    const uint32_t lc = ch - sg.chunk0;
    const uint32_t t0 = sg.tile0 + lc * kChunk;
    const uint32_t tend = sg.tile0 + sg.ntiles;
    const uint32_t t1 = t0 + kChunk < tend ? t0 + kChunk : tend;
    const uint32_t nb = sg.nbk;
    for (uint32_t b = threadIdx.x; b < nb; b += 256) {
        uint32_t s = 0;
        for (uint32_t t = t0; t < t1; ++t) s += a.C[(size_t)t * kNbStride + b];
        a.P[(size_t)ch * kNbStride + b] = s;
    }
}

__global__ __launch_bounds__(256) void k_scan_chunks(LevelArgs a)
{
    scan_chunks_item(a, blockIdx.x, a.nsegs);
}

__global__ __launch_bounds__(256) void k_scan_chunks_ds(LevelArgs a)
{
    const uint32_t ns = ds_nsegs(a), n = a.dims->chunks;
    for (uint32_t ch = blockIdx.x; ch < n; ch += gridDim.x) scan_chunks_item(a, ch, ns);
}

__device__ __forceinline__ void scan_buckets_item(const LevelArgs& a, uint32_t blk)
{
    __shared__ uint32_t part[16][64];
    const uint32_t sid = blk / kBucketGroups;
    const uint32_t bg = blk % kBucketGroups;
    const Seg sg = a.segs[sid];
    const uint32_t nb = sg.nbk;
    if (bg * 64 >= nb) return;  // uniform over the block
    const uint32_t col = threadIdx.x & 63u, row = threadIdx.x >> 6;
    const uint32_t b = bg * 64 + col;
    const uint32_t nch = (sg.ntiles + kChunk - 1) / kChunk;
    const uint32_t per = (nch + 15) / 16;
    const uint32_t c0 = row * per;
    const uint32_t c1 = c0 + per < nch ? c0 + per : nch;
    uint32_t s = 0;
    if (b < nb)
        for (uint32_t c = c0; c < c1; ++c) s += a.P[(size_t)(sg.chunk0 + c) * kNbStride + b];
    part[row][col] = s;
    __syncthreads();
    uint32_t pre = 0;
    for (uint32_t r = 0; r < row; ++r) pre += part[r][col];
    if (b < nb) {
        for (uint32_t c = c0; c < c1; ++c) {
            uint32_t* p = a.P + (size_t)(sg.chunk0 + c) * kNbStride + b;
            const uint32_t x = *p;
            *p = pre;
            pre += x;
        }
        if (row == 15) a.tot[(size_t)sid * kNbStride + b] = pre;
    }
}

__global__ __launch_bounds__(1024) void k_scan_buckets(LevelArgs a)
{
    scan_buckets_item(a, blockIdx.x);
}

__global__ __launch_bounds__(1024) void k_scan_buckets_ds(LevelArgs a)
{
    const uint32_t n = ds_nsegs(a) * kBucketGroups;
    for (uint32_t blk = blockIdx.x; blk < n; blk += gridDim.x) {
        scan_buckets_item(a, blk);
        __syncthreads();
    }
}

__device__ __forceinline__ void scan_offsets_item(const LevelArgs& a, uint32_t sid)
{
    __shared__ uint32_t tmp[20];
    const Seg sg = a.segs[sid];
    const uint32_t nb = sg.nbk;
    const uint32_t b0 = 2 * threadIdx.x, b1 = b0 + 1;
    const uint32_t v0 = b0 < nb ? a.tot[(size_t)sid * kNbStride + b0] : 0u;
    const uint32_t v1 = b1 < nb ? a.tot[(size_t)sid * kNbStride + b1] : 0u;
    uint32_t total = 0;
    const uint32_t base = block_excl_scan<1024>(v0 + v1, tmp, &total);
    uint32_t* bs = a.bstart + (size_t)sid * (kNbStride + 1);
    if (b0 < nb) bs[b0] = sg.start + base;
    if (b1 < nb) bs[b1] = sg.start + base + v0;
    if (threadIdx.x == 0) {
        // collect-reduce keeps heavy records out of the buckets (one slot each)
        bs[nb] = sg.start + total;
        if (a.reduce ? total > sg.len : total != sg.len) atomicOr(&a.info->status, kStatusSizeMismatch);
    }
}

__global__ __launch_bounds__(1024) void k_scan_offsets(LevelArgs a)
{
    scan_offsets_item(a, blockIdx.x);
}

__global__ __launch_bounds__(1024) void k_scan_offsets_ds(LevelArgs a)
{
    const uint32_t n = ds_nsegs(a);
    for (uint32_t sid = blockIdx.x; sid < n; sid += gridDim.x) {
        scan_offsets_item(a, sid);
        __syncthreads();
    }
}

__device__ __forceinline__ void scan_fill_item(const LevelArgs& a, uint32_t ch, uint32_t nsegs)
{
    const uint32_t sid = find_by_chunk(a.segs, nsegs, ch);
    const Seg sg = a.segs[sid];
    const uint32_t lc = ch - sg.chunk0;
    const uint32_t t0 = sg.tile0 + lc * kChunk;
    const uint32_t tend = sg.tile0 + sg.ntiles;
    const uint32_t t1 = t0 + kChunk < tend ? t0 + kChunk : tend;
    const uint32_t nb = sg.nbk;
    const uint32_t* bs = a.bstart + (size_t)sid * (kNbStride + 1);
    for (uint32_t b = threadIdx.x; b < nb; b += 256) {
        uint32_t x = bs[b] + a.P[(size_t)ch * kNbStride + b];
        for (uint32_t t = t0; t < t1; ++t) {
            uint32_t* p = a.C + (size_t)t * kNbStride + b;
            const uint32_t c = *p;
            *p = x;
            x += c;
        }
    }
}

__global__ __launch_bounds__(256) void k_scan_fill(LevelArgs a)
{
    scan_fill_item(a, blockIdx.x, a.nsegs);
}

__global__ __launch_bounds__(256) void k_scan_fill_ds(LevelArgs a)
{
    const uint32_t ns = ds_nsegs(a), n = a.dims->chunks;
    for (uint32_t ch = blockIdx.x; ch < n; ch += gridDim.x) scan_fill_item(a, ch, ns);
}

// ================================================================ Step 2c
// Distribution (Section 3.2): each subarray, in order, moves every record to
// T[X[i][id]++].  One block per subarray walks it in sub-tiles of W*64*E
// records.  Bucket ids come from the counting pass, so no hashing or table
// lookup is repeated here.  Each wave ranks its contiguous chunk stably
// (ballot match plus per-wave LDS counters), the block turns ranks into
// bucket-grouped LDS positions, and the staged sub-tile is written out so
// that consecutive threads write consecutive addresses of a bucket's run.
// Keys go first, then values through the same staging buffer; the next
// sub-tile's loads are issued before the current one is ranked.  Buckets that
// are final (heavy, single record, or all hash bits used) go to fin_* -- the
// output -- when that is safe, so they are never copied again.

__device__ __forceinline__ bool bucket_is_final(bool one_key_bucket, uint32_t sz, bool all_bits_used)
{
    return one_key_bucket || sz <= 1 || all_bits_used;
}

// RED = 0: semisort; RED = 1: collect-reduce (heavy records are summed in
// LDS and added to the subproblem's heavy sums, light records move); RED = 2:
// histogram (as 1 with every value 1 and no value array).
template <typename V, int W, int E, int RED, typename K>
__device__ __forceinline__ void distribute_item(const LevelArgs& a, uint32_t t, uint32_t nsegs, uint32_t tile)
{
    // Every global load and store in the sub-tile loop is issued
    // unconditionally (clamped 32-bit load offsets from the sub-tile's start,
    // a sink address for lanes without a record to write): with no branches
    // around memory instructions the compiler can count outstanding accesses
    // and wait only for the ones it needs instead of draining all stores
    // before the next loads are used.  Each bucket's output range for the
    // sub-tile is checked once against its subproblem; a sub-tile with a bad
    // range writes nothing and raises the status.
    constexpr int BS = W * 64;
    constexpr int SUB = BS * E;
    __shared__ uint32_t gbase[kNbStride];      // bit 31: bucket goes to fin_*
    __shared__ uint32_t lst[kNbStride + 1];
    // output position - stage slot (31 bits, wrapping) | bit 31 of gbase
    __shared__ uint32_t dl[kNbStride];
    __shared__ uint32_t sh_bad;
    __shared__ uint16_t wc[W * kNbStride];
    constexpr int KW = sizeof(KReg<K>) / 8;  // words per key in registers
    __shared__ uint64_t stage[SUB * KW];
    __shared__ uint16_t stage_b[SUB];
    __shared__ uint32_t tmp[20];
    __shared__ unsigned long long hs[RED ? kNbStride : 1];
    __shared__ uint8_t finl[kNbStride];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, w = tid >> 6;
    const uint32_t sid = find_by_tile(a.segs, nsegs, t);
    const Seg sg = a.segs[sid];
    const uint32_t lt = t - sg.tile0;
    const uint64_t r0 = (uint64_t)sg.start + (uint64_t)lt * tile;
    const uint64_t send = (uint64_t)sg.start + sg.len;
    const uint64_t r1 = r0 + tile < send ? r0 + tile : send;
    const uint64_t rlast = r1 - 1;
    const uint32_t nL = 1u << sg.nl_bits;
    const uint32_t nb = sg.nbk;
    const uint32_t nbits = 32 - __clz(nb - 1);
    const bool split = a.fin_keys != a.dst_keys;
    const bool all_bits = a.ordered == 0 && (uint32_t)sg.shift + sg.nl_bits >= KeyTraits<K>::hash_bits;
    const uint32_t* bsz = a.bstart + (size_t)sid * (kNbStride + 1);
    const uint8_t* fin = a.bfin + (size_t)sid * kNbStride;
    const V* src_vals = (const V*)a.src_vals;
    V* dst_vals = (V*)a.dst_vals;
    V* fin_vals = (V*)a.fin_vals;
    V* stage_v = (V*)stage;
    const uint32_t per = (nb + BS - 1) / BS;  // buckets per thread in the scans
    const uint32_t pb0 = tid * per;
    const bool fillk = RED == 0 && a.fill_heavy != 0;

    for (uint32_t b = tid; b < nb; b += BS) {
        uint32_t g = a.C[(size_t)t * kNbStride + b];
        if (split && bucket_is_final(fin[b] != 0, bsz[b + 1] - bsz[b], all_bits)) g |= 0x80000000u;
        gbase[b] = g;
        finl[b] = fin[b];
        if constexpr (RED != 0) hs[b] = RED == 1 ? red_identity(a.rop) : 0ull;
    }
    for (uint32_t i = tid; i < W * nb; i += BS) wc[i] = 0;

    // keys and bucket ids are loaded one sub-tile ahead; values at the top of
    // their own iteration (needed only after the ranking)
    const uint32_t lofs = w * 64 * E + lane;  // this lane's first offset in a sub-tile
    K* sink_k = (K*)a.sink + lane;
    V* sink_v = (V*)(a.sink + lane);
    const uint64_t kdiff = (uint64_t)a.fin_keys - (uint64_t)a.dst_keys;
    const uint64_t vdiff = (uint64_t)fin_vals - (uint64_t)dst_vals;
    // Keys are not needed for records of one-key buckets whose keys k_fill
    // writes, nor for the heavy records of the reduction forms (they stay):
    // their key loads read a sink line (an L2 hit) instead of the input, so
    // key loads wait for the bucket ids, which are loaded first.
    auto skip_key = [&](uint32_t b) -> bool {
        if constexpr (RED != 0) return finl[b] != 0;
        else return fillk && finl[b] != 0;
    };
    KReg<K> kn[E];
    uint16_t bn[E];
    {
        const uint16_t* bs = a.bids + r0;
        const uint32_t lim = (uint32_t)(rlast - r0 < SUB ? rlast - r0 : SUB);
#pragma unroll
        for (int e = 0; e < E; ++e) bn[e] = bs[min(lofs + e * 64u, lim)];
    }
    if (tid == 0) sh_bad = 0;
    __syncthreads();
    {
        const K* ks = (const K*)a.src_keys + r0;
        const uint32_t lim = (uint32_t)(rlast - r0 < SUB ? rlast - r0 : SUB);
#pragma unroll
        for (int e = 0; e < E; ++e) kn[e] = kload(skip_key(bn[e]) ? sink_k : ks + min(lofs + e * 64u, lim));
    }

    bool out_of_range = false;
    for (uint64_t sub = r0; sub < r1; sub += SUB) {
        KReg<K> k[E];
        V v[E];
        uint32_t bk[E], pos[E];
        const uint32_t left = (uint32_t)(r1 - sub < 2 * SUB ? r1 - sub : 2 * SUB);  // records from sub on
        {
            const V* vs = src_vals + sub;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const uint32_t o = min(lofs + e * 64u, left - 1);
                if constexpr (RED == 2) v[e] = (V)1;
                else v[e] = vs[o];
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            k[e] = kn[e];
            bk[e] = bn[e];
        }
        {
            // bucket ids of the next sub-tile (the last iteration re-reads its
            // own, clamped); its keys are loaded once these have arrived
            const uint16_t* bs = a.bids + sub;
#pragma unroll
            for (int e = 0; e < E; ++e) bn[e] = bs[min(lofs + SUB + e * 64u, left - 1)];
        }
        uint16_t* wcw = wc + w * nb;
        bool mv[E];  // this record moves (heavy records of collect-reduce stay)
#pragma unroll
        for (int e = 0; e < E; ++e) {
            mv[e] = lofs + e * 64u < left;
            if constexpr (RED != 0) {
                if (mv[e] && finl[bk[e]]) {
                    if constexpr (RED == 1) red_atomic(a.rop, &hs[bk[e]], (unsigned long long)v[e]);
                    else atomicAdd(&hs[bk[e]], (unsigned long long)v[e]);
                    mv[e] = false;
                }
            }
        }
        wave_rank_all<E>(bk, mv, nbits, wcw, pos);
        {
            const K* ks = (const K*)a.src_keys + sub;
#pragma unroll
            for (int e = 0; e < E; ++e)
                kn[e] = kload(skip_key(bn[e]) ? sink_k : ks + min(lofs + SUB + e * 64u, left - 1));
        }
        __syncthreads();

        // per bucket: exclusive prefix over waves, sub-tile total, and the
        // exclusive scan of the totals over buckets (contiguous pieces per thread)
        uint32_t s = 0;
        for (uint32_t j = 0; j < per; ++j) {
            const uint32_t b = pb0 + j;
            if (b < nb) {
                uint32_t run = 0;
#pragma unroll 4
                for (int ww = 0; ww < W; ++ww) {
                    const uint32_t c = wc[ww * nb + b];
                    wc[ww * nb + b] = (uint16_t)run;
                    run += c;
                }
                lst[b] = run;  // total for now
                s += run;
            }
        }
        uint32_t tot = 0;
        uint32_t run = block_excl_scan<BS>(s, tmp, &tot);
        bool bad = false;
        for (uint32_t j = 0; j < per; ++j) {
            const uint32_t b = pb0 + j;
            if (b < nb) {
                const uint32_t c = lst[b];
                const uint32_t g = gbase[b];
                const uint32_t p = g & 0x7FFFFFFFu;
                // [p, p + c) must lie inside the subproblem
                bad |= c != 0 && (c > sg.len || p - sg.start > sg.len - c);
                lst[b] = run;
                dl[b] = ((p - run) & 0x7FFFFFFFu) | (g & 0x80000000u);
                run += c;
            }
        }
        if (bad) sh_bad = 1;
        if (tid == 0) lst[nb] = tot;
        __syncthreads();

        // stage keys in bucket order
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (mv[e]) {
                const uint32_t b = bk[e];
                const uint32_t p = lst[b] + wc[w * nb + b] + pos[e];
                pos[e] = p;
                ((KReg<K>*)stage)[p] = k[e];
                // bit 15: the key is not stored (one-key bucket, filled later)
                stage_b[p] = (uint16_t)(b | ((fillk && finl[b]) ? 0x8000u : 0u));
            }
        }
        __syncthreads();
        const uint32_t m = sh_bad ? 0u : lst[nb];  // a bad range: write nothing
        out_of_range |= sh_bad != 0;
        uint32_t dest[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t j = tid + e * BS;
            const uint32_t jj = j < m ? j : 0u;
            const uint32_t sb = stage_b[jj];
            const uint32_t x = dl[__builtin_amdgcn_ubfe(sb, 0, 15)];
            const uint32_t d = (jj + x) & 0x7FFFFFFFu;
            dest[e] = j < m ? (d | (x & 0x80000000u)) : 0xFFFFFFFFu;
            // dst_keys, or fin_keys when bit 31 is set: a masked difference
            // (kept opaque, or the compiler turns it back into a select that
            // copies both uniform pointers into VGPRs)
            uint32_t msk = (uint32_t)((int32_t)x >> 31);
            __asm__("" : "+v"(msk));
            const uint64_t sel = ((uint64_t)msk << 32) | msk;
            K* out = (K*)((char*)a.dst_keys + (kdiff & sel)) + d;
            // bit 15: the key is not stored (one-key bucket, filled later)
            *(j < m && !(sb >> 15) ? out : sink_k) = knarrow<K>(((const KReg<K>*)stage)[jj]);
        }
        for (uint32_t i = tid; i < W * nb; i += BS) wc[i] = 0;
        __syncthreads();
        if constexpr (RED != 2) {
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (mv[e]) stage_v[pos[e]] = v[e];
            __syncthreads();
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const uint32_t j = tid + e * BS;
                const uint32_t dd = dest[e];
                uint32_t msk = (uint32_t)((int32_t)dd >> 31);
                __asm__("" : "+v"(msk));
                const uint64_t sel = ((uint64_t)msk << 32) | msk;
                V* out = (V*)((char*)dst_vals + (vdiff & sel)) + (dd & 0x7FFFFFFFu);
                *(dd != 0xFFFFFFFFu ? out : sink_v) = stage_v[j < m ? j : 0u];
            }
            __syncthreads();
        }
        for (uint32_t j = 0; j < per; ++j) {
            const uint32_t b = pb0 + j;
            if (b < nb) gbase[b] += lst[b + 1] - lst[b];
        }
    }
    if constexpr (RED != 0) {
        __syncthreads();
        for (uint32_t b = tid; b < nb; b += BS)
            if (finl[b] && hs[b] != (RED == 1 ? red_identity(a.rop) : 0ull))  // the identity changes nothing
                red_atomic(RED == 1 ? a.rop : 0u, &a.hsum[(size_t)sid * kHeavyMax + (b - nL)], hs[b]);
    }
    if (out_of_range) atomicOr(&a.info->status, kStatusScatterRange);
}

template <typename V, int W, int E, int RED, typename K = uint64_t>
__global__ __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_distribute(LevelArgs a)
{
    distribute_item<V, W, E, RED, K>(a, xcd_remap(blockIdx.x, gridDim.x), a.nsegs, a.tile);
}

template <typename V, int W, int E, int RED>
__global__ __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_distribute_ds(LevelArgs a)
{
    __shared__ uint32_t sh_t;
    const uint32_t ns = ds_nsegs(a), n = a.dims->tiles, tile = a.dims->tile;
    for (uint32_t t = xcd_queue_next(a.q + 8, n, &sh_t); t < n; t = xcd_queue_next(a.q + 8, n, &sh_t))
        distribute_item<V, W, E, RED, uint64_t>(a, t, ns, tile);
}

// Direct form of the distribution: the same stable ranking, but every record
// is written straight from registers to its destination, without staging
// the sub-tile in LDS.  Lanes of a wave that share a bucket in a round hold
// consecutive ranks, so heavy buckets still produce contiguous stores; the L2
// merges the short runs of light buckets.  LDS holds only the per-wave
// counters (double-buffered) and the bucket bases, so several blocks share a
// CU and one block's ranking overlaps another's stores.
template <typename V, int W, int E, int WPE>
__global__ __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void k_distribute_direct(LevelArgs a)
{
    constexpr int BS = W * 64;
    constexpr int SUB = BS * E;
    __shared__ uint32_t gbase[kNbStride];      // bit 31: bucket goes to fin_*
    __shared__ uint32_t ptot[kNbStride];       // previous sub-tile's bucket totals
    __shared__ uint16_t wc[2][W * kNbStride];

    const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, w = tid >> 6;
    const uint32_t sid = find_by_tile(a.segs, a.nsegs, t);
    const Seg sg = a.segs[sid];
    const uint32_t lt = t - sg.tile0;
    const uint64_t r0 = (uint64_t)sg.start + (uint64_t)lt * a.tile;
    const uint64_t send = (uint64_t)sg.start + sg.len;
    const uint64_t r1 = r0 + a.tile < send ? r0 + a.tile : send;
    const uint64_t rlast = r1 - 1;
    const uint32_t nb = sg.nbk;
    const uint32_t nbits = 32 - __clz(nb - 1);
    const bool split = a.fin_keys != a.dst_keys;
    const bool all_bits = a.ordered == 0 && (uint32_t)sg.shift + sg.nl_bits >= 64;
    const uint32_t* bsz = a.bstart + (size_t)sid * (kNbStride + 1);
    const uint8_t* fin = a.bfin + (size_t)sid * kNbStride;
    const V* src_vals = (const V*)a.src_vals;
    V* dst_vals = (V*)a.dst_vals;
    V* fin_vals = (V*)a.fin_vals;
    uint64_t* sink_k = a.sink + lane;
    V* sink_v = (V*)(a.sink + lane);
    const uint32_t per = (nb + BS - 1) / BS;  // buckets per thread in the scans
    const uint32_t pb0 = tid * per;

    for (uint32_t b = tid; b < nb; b += BS) {
        uint32_t g = a.C[(size_t)t * kNbStride + b];
        if (split && bucket_is_final(fin[b] != 0, bsz[b + 1] - bsz[b], all_bits)) g |= 0x80000000u;
        gbase[b] = g;
        ptot[b] = 0;
    }
    for (uint32_t i = tid; i < W * nb; i += BS) {
        wc[0][i] = 0;
        wc[1][i] = 0;
    }

    uint16_t bn[E];
    {
        const uint64_t bi = r0 + (uint64_t)w * 64 * E + lane;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            uint64_t i = bi + (uint64_t)e * 64;
            i = i < rlast ? i : rlast;
            bn[e] = a.bids[i];
        }
    }
    __syncthreads();

    bool out_of_range = false;
    uint32_t cur = 0;
    for (uint64_t sub = r0; sub < r1; sub += SUB, cur ^= 1u) {
        uint64_t k[E];
        V v[E];
        uint32_t bk[E], pos[E];
        const uint64_t base_i = sub + (uint64_t)w * 64 * E + lane;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            uint64_t i = base_i + (uint64_t)e * 64;
            i = i < rlast ? i : rlast;
            k[e] = a.src_keys[i];
            v[e] = src_vals[i];
            bk[e] = bn[e];
        }
        {
            const uint64_t bi = base_i + SUB;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                uint64_t i = bi + (uint64_t)e * 64;
                i = i < rlast ? i : rlast;
                bn[e] = a.bids[i];
            }
        }
        uint16_t* wcc = wc[cur];
        uint16_t* wcw = wcc + w * nb;
#pragma unroll
        for (int e = 0; e < E; ++e) pos[e] = wave_rank(bk[e], base_i + (uint64_t)e * 64 < r1, nbits, wcw);
        __syncthreads();

        // The other counter buffer was last read by the previous sub-tile's
        // stores, which every thread finished before the barrier above; clear
        // it for the next sub-tile (the barrier below orders it before use).
        for (uint32_t i = tid; i < W * nb; i += BS) wc[cur ^ 1][i] = 0;
        // per bucket: advance the base past the previous sub-tile, then turn
        // the wave counters into bucket-local prefixes
        for (uint32_t j = 0; j < per; ++j) {
            const uint32_t b = pb0 + j;
            if (b < nb) {
                gbase[b] += ptot[b];
                uint32_t run = 0;
#pragma unroll 4
                for (int ww = 0; ww < W; ++ww) {
                    const uint32_t c = wcc[ww * nb + b];
                    wcc[ww * nb + b] = (uint16_t)run;
                    run += c;
                }
                ptot[b] = run;
            }
        }
        __syncthreads();

#pragma unroll
        for (int e = 0; e < E; ++e) {
            const bool valid = base_i + (uint64_t)e * 64 < r1;
            const uint32_t b = bk[e];
            const uint32_t dd = gbase[b] + wcc[w * nb + b] + pos[e];
            const uint32_t d = dd & 0x7FFFFFFFu;
            const bool in_range = d - sg.start < sg.len;
            out_of_range |= valid && !in_range;
            const bool ok = valid && in_range;
            uint64_t* ko = (dd >> 31) ? a.fin_keys : a.dst_keys;
            V* vo = (dd >> 31) ? fin_vals : dst_vals;
            *(ok ? ko + d : sink_k) = k[e];
            *(ok ? vo + d : sink_v) = v[e];
        }
    }
    if (out_of_range) atomicOr(&a.info->status, kStatusScatterRange);
}

// ================================================================ Step 3 planning
// After a level's distribution, every bucket of every subproblem becomes one
// of: a subproblem of the next level (light, >= alpha records: the recursive
// call of Algorithm 1), a base-case job (light, 2 .. alpha-1 records), a copy
// job (a bucket that is already final but sits in T, Section 3.4), or nothing.
// Heavy buckets are final (Section 3.3).  Base-case jobs are sorted into
// capacity classes; appends are aggregated per block.

struct PlanArgs {
    const Seg* segs;
    uint32_t nsegs;
    const uint32_t* bstart;
    Seg* next;
    uint32_t next_cap;
    Job* jobs;          // kJobClasses lists: list c holds job_capc[c] entries from job_base[c]
    uint64_t job_base[kJobClasses];
    uint32_t job_capc[kJobClasses];
    LevelInfo* info;
    uint32_t alpha;
    uint32_t finals_in_out;  // final buckets were written to the output by the distribution
    uint32_t ordered;        // splitter buckets: no hash bits are consumed
    const uint8_t* bfin;     // [nsegs][kNbStride] one-key bucket flags
    uint32_t reduce;         // collect-reduce: heavy buckets are done, one-key buckets are summed
    uint32_t fill;           // one-key final buckets in the output get key-fill jobs
    const uint64_t* bkey;    // [nsegs][kNbStride] keys of one-key buckets
    FillJob* fills;
    uint32_t fill_cap;
    uint32_t hash_bits = 64;  // hash bits the levels can consume (128 for 128-bit keys)
    // device-sized levels: the current level's subproblem count is read from
    // dims (bounded by cur_cap) instead of nsegs
    const LevelInfo* dims;
    uint32_t cur_cap;
};

struct PlanCount {
    uint32_t seg;
    uint32_t job[kJobClasses];
    uint32_t fill;
    uint32_t rec;
    uint32_t frec;
};

// What bucket b of subproblem sg turns into; with emit, write it at the
// cursors (seg_at, job_at[class]).
__device__ __forceinline__ void plan_bucket(const PlanArgs& p, uint32_t sidx, const Seg& sg, uint32_t b,
                                            uint32_t nL, PlanCount& cnt, bool emit, uint32_t* seg_at,
                                            uint32_t* job_at, uint32_t* fill_at)
{
    const uint32_t* bs = p.bstart + (size_t)sidx * (kNbStride + 1);
    const uint32_t st = bs[b];
    const uint32_t sz = bs[b + 1] - st;
    if (sz == 0) return;
    const uint32_t shift2 = p.ordered ? 0u : (uint32_t)sg.shift + sg.nl_bits;
    const bool all_bits_used = shift2 >= p.hash_bits;
    if (p.reduce) {
        // heavy bucket: its result was written with the level; a bucket of one
        // record, or of one hash value (one key: the hash is a bijection),
        // becomes a sum job in the copy class
        if (p.bfin[(size_t)sidx * kNbStride + b]) return;
        if (sz == 1 || all_bits_used) {
            if (emit) {
                if (job_at[kCopyClass] < p.job_capc[kCopyClass]) p.jobs[p.job_base[kCopyClass] + job_at[kCopyClass]] = Job{st, sz};
                ++job_at[kCopyClass];
            }
            ++cnt.job[kCopyClass];
            cnt.rec += sz;
            return;
        }
    } else if (bucket_is_final(p.bfin[(size_t)sidx * kNbStride + b] != 0, sz, all_bits_used)) {
        if (p.finals_in_out) {  // already in place, except the keys of one-key buckets
            if (p.fill && p.bfin[(size_t)sidx * kNbStride + b]) {
                const uint64_t key = p.bkey[(size_t)sidx * kNbStride + b];
                for (uint32_t o = 0; o < sz; o += kFillChunk) {
                    const uint32_t l = sz - o < kFillChunk ? sz - o : kFillChunk;
                    if (emit) {
                        if (*fill_at < p.fill_cap) p.fills[*fill_at] = FillJob{st + o, l, key};
                        ++*fill_at;
                    }
                    ++cnt.fill;
                }
                cnt.frec += sz;
            }
            return;
        }
        for (uint32_t o = 0; o < sz; o += kCopyChunk) {
            const uint32_t l = sz - o < kCopyChunk ? sz - o : kCopyChunk;
            if (emit && job_at[kCopyClass] < p.job_capc[kCopyClass])
                p.jobs[p.job_base[kCopyClass] + job_at[kCopyClass]] = Job{st + o, l};
            if (emit) ++job_at[kCopyClass];
            ++cnt.job[kCopyClass];
        }
        cnt.rec += sz;
        return;
    }
    if (sz >= p.alpha) {
        if (emit) {
            if (*seg_at < p.next_cap) {
                Seg ns;
                ns.start = st;
                ns.len = sz;
                ns.ibase = sg.ibase;
                ns.tile0 = ns.chunk0 = ns.ntiles = 0;
                ns.nl_bits = (uint8_t)choose_nl(sz, p.alpha, kLightBitsMax, shift2, p.hash_bits);
                ns.shift = (uint8_t)shift2;
                ns.nbk = 0;
                ns.nheavy = 0;
                ns.hlog2 = 0;
                p.next[*seg_at] = ns;
            }
            ++*seg_at;
        }
        ++cnt.seg;
        return;
    }
    const int c = base_class(sz);
    if (emit) {
        if (job_at[c] < p.job_capc[c]) p.jobs[p.job_base[c] + job_at[c]] = Job{st, sz};
        ++job_at[c];
    }
    ++cnt.job[c];
    cnt.rec += sz;
}

__device__ __forceinline__ void plan_item(const PlanArgs& p, uint32_t sidx)
{
    __shared__ uint32_t tmp[20];
    __shared__ uint32_t sh_base[kJobClasses + 2];
    const Seg sg = p.segs[sidx];
    const uint32_t nL = 1u << sg.nl_bits;
    const uint32_t nb = sg.nbk;
    PlanCount cnt{};
    uint32_t dummy_s = 0, dummy_j[kJobClasses] = {}, dummy_f = 0;
    for (uint32_t b = threadIdx.x; b < nb; b += 256)
        plan_bucket(p, sidx, sg, b, nL, cnt, false, &dummy_s, dummy_j, &dummy_f);
    uint32_t tot = 0;
    uint32_t seg_at = block_excl_scan<256>(cnt.seg, tmp, &tot);
    if (threadIdx.x == 0) sh_base[kJobClasses] = tot ? atomicAdd(&p.info->nsegs, tot) : 0u;
    uint32_t job_at[kJobClasses];
#pragma unroll
    for (int c = 0; c < kJobClasses; ++c) {
        job_at[c] = block_excl_scan<256>(cnt.job[c], tmp, &tot);
        if (threadIdx.x == 0) sh_base[c] = tot ? atomicAdd(&p.info->njobs[c], tot) : 0u;
    }
    uint32_t fill_at = block_excl_scan<256>(cnt.fill, tmp, &tot);
    if (threadIdx.x == 0) sh_base[kJobClasses + 1] = tot ? atomicAdd(&p.info->nfills, tot) : 0u;
    uint32_t rtot = 0;
    (void)block_excl_scan<256>(cnt.rec, tmp, &rtot);
    if (threadIdx.x == 0 && rtot) atomicAdd(&p.info->job_records, (unsigned long long)rtot);
    (void)block_excl_scan<256>(cnt.frec, tmp, &rtot);
    if (threadIdx.x == 0 && rtot) atomicAdd(&p.info->fill_records, (unsigned long long)rtot);
    __syncthreads();
    seg_at += sh_base[kJobClasses];
    fill_at += sh_base[kJobClasses + 1];
#pragma unroll
    for (int c = 0; c < kJobClasses; ++c) job_at[c] += sh_base[c];
    PlanCount again{};
    for (uint32_t b = threadIdx.x; b < nb; b += 256)
        plan_bucket(p, sidx, sg, b, nL, again, true, &seg_at, job_at, &fill_at);
}

__global__ __launch_bounds__(256) void k_plan(PlanArgs p)
{
    plan_item(p, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_plan_ds(PlanArgs p)
{
    const uint32_t c = p.dims->nsegs, n = c < p.cur_cap ? c : p.cur_cap;
    for (uint32_t sidx = blockIdx.x; sidx < n; sidx += gridDim.x) {
        plan_item(p, sidx);
        __syncthreads();
    }
}

// Prefix over the next level's subproblems: subarray size for the level,
// then first tile and first scan chunk of every subproblem.  One block.
__global__ __launch_bounds__(1024) void k_seg_prefix(Seg* segs, uint32_t cap, LevelInfo* info,
                                                     uint32_t tmin, uint32_t tmax)
{
    __shared__ uint32_t tmp[20];
    __shared__ unsigned long long sh_total;
    const uint32_t n = info->nsegs < cap ? info->nsegs : cap;
    if (threadIdx.x == 0) sh_total = 0;
    __syncthreads();
    unsigned long long mine = 0;
    for (uint32_t i = threadIdx.x; i < n; i += 1024) mine += segs[i].len;
    atomicAdd(&sh_total, mine);
    __syncthreads();
    const uint32_t tile = choose_tile(sh_total, tmin, tmax);
    uint32_t run_t = 0, run_c = 0;
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        uint32_t nt = 0, nc = 0;
        if (i < n) {
            nt = (segs[i].len + tile - 1) / tile;
            nc = (nt + kChunk - 1) / kChunk;
        }
        uint32_t tt = 0, tc = 0;
        const uint32_t ot = block_excl_scan<1024>(nt, tmp, &tt);
        const uint32_t oc = block_excl_scan<1024>(nc, tmp, &tc);
        if (i < n) {
            segs[i].tile0 = run_t + ot;
            segs[i].chunk0 = run_c + oc;
            segs[i].ntiles = nt;
        }
        run_t += tt;
        run_c += tc;
    }
    if (threadIdx.x == 0) {
        info->tiles = run_t;
        info->chunks = run_c;
        info->tile = tile;
        info->records = sh_total;
    }
}

// ---------------------------------------------------------------- graph transpose
// Section 5 (graph transposing): for a CSR graph the transpose is a stable
// semisort of the edges by their other endpoint.  These kernels turn the CSR
// into (other endpoint, first endpoint) records and the sorted endpoints back
// into row offsets; the sort in between is semisort_<.

constexpr uint32_t kExpandEdges = 4096;  // edges per block of k_csr_expand

// Last row r in [lo, hi] with offs[r] <= e (offs non-decreasing over the range).
__device__ __forceinline__ uint32_t csr_row_of(const uint64_t* offs, uint32_t lo, uint32_t hi, uint64_t e)
{
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        if (offs[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Offsets must not decrease (the ends are checked on the host).
__global__ __launch_bounds__(256) void k_csr_check(const uint64_t* offs, uint32_t nv, LevelInfo* info)
{
    bool bad = false;
    for (uint64_t u = (uint64_t)blockIdx.x * 256 + threadIdx.x; u < nv; u += (uint64_t)gridDim.x * 256)
        bad |= offs[u + 1] < offs[u];
    if (bad) atomicOr(&info->status, kStatusBadGraph);
}

// Edge e of row u becomes the record (key cols[e], value u).  A block takes
// kExpandEdges consecutive edges; its first and last rows are found once over
// all rows, each edge's row then inside that range.
__global__ __launch_bounds__(256) void k_csr_expand(const uint64_t* offs, const uint32_t* cols, uint32_t nv,
                                                    uint64_t ne, uint64_t* keys, uint32_t* vals, LevelInfo* info)
{
    __shared__ uint32_t sh_r[2];
    const uint64_t s = (uint64_t)blockIdx.x * kExpandEdges;
    const uint64_t t = s + kExpandEdges < ne ? s + kExpandEdges : ne;
    if (threadIdx.x < 2) sh_r[threadIdx.x] = csr_row_of(offs, 0, nv - 1, threadIdx.x ? t - 1 : s);
    __syncthreads();
    const uint32_t r0 = sh_r[0], r1 = sh_r[1] < r0 ? r0 : sh_r[1];
    bool bad = false;
    for (uint64_t e = s + threadIdx.x; e < t; e += 256) {
        const uint32_t v = cols[e];
        const uint32_t u = csr_row_of(offs, r0, r1, e);
        bad |= v >= nv || offs[u] > e || offs[u + 1] <= e;
        keys[e] = v;
        vals[e] = u;
    }
    if (bad) atomicOr(&info->status, kStatusBadGraph);
}

// Row offsets of the transpose from the sorted endpoints: the first position
// of every endpoint value v goes to out[v] (out[] starts at ~0, out[nv] = ne),
// then a suffix minimum gives the vertices without edges the next start.
__global__ __launch_bounds__(256) void k_csr_starts(const uint64_t* skeys, uint64_t ne, uint32_t nv, uint64_t* out,
                                                    LevelInfo* info)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < ne; i += (uint64_t)gridDim.x * 256) {
        const uint64_t k = skeys[i];
        if (k >= nv) {
            atomicOr(&info->status, kStatusBadGraph);
            continue;
        }
        if (i == 0 || skeys[i - 1] != k) out[k] = i;
    }
}

// out[v] = ~0 for v < nv (no start yet), out[nv] = ne.
__global__ __launch_bounds__(256) void k_csr_init(uint64_t* out, uint32_t nv, uint64_t ne)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i <= nv; i += (uint64_t)gridDim.x * 256)
        out[i] = i == nv ? ne : ~0ull;
}

constexpr uint32_t kMinChunk = 4096;  // entries per block of the suffix-minimum passes

__device__ __forceinline__ unsigned long long block_min_u64(unsigned long long x, unsigned long long* tmp)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    const uint32_t w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63u) == 0) tmp[w] = x;
    __syncthreads();
    unsigned long long m = tmp[0];
    for (uint32_t i = 1; i < nw; ++i) m = tmp[i] < m ? tmp[i] : m;
    return m;
}

// Pass 1: the minimum of every chunk of out[0 .. n).
__global__ __launch_bounds__(256) void k_min_chunks(const uint64_t* out, uint64_t n, uint64_t* cmin)
{
    __shared__ unsigned long long tmp[4];
    const uint64_t s = (uint64_t)blockIdx.x * kMinChunk;
    unsigned long long m = ~0ull;
    for (uint64_t i = s + threadIdx.x; i < s + kMinChunk && i < n; i += 256) m = out[i] < m ? out[i] : m;
    m = block_min_u64(m, tmp);
    if (threadIdx.x == 0) cmin[blockIdx.x] = m;
}

// Pass 2 (one block): cmin[b] becomes the minimum over the chunks after b.
__global__ __launch_bounds__(1024) void k_min_carry(uint64_t* cmin, uint32_t nb)
{
    __shared__ unsigned long long buf[1024];
    __shared__ unsigned long long sh_carry;
    if (threadIdx.x == 0) sh_carry = ~0ull;
    __syncthreads();
    // walk the chunk minima from the end, 1024 at a time
    for (int64_t base = (int64_t)nb - 1024; base > -1024; base -= 1024) {
        const int64_t i = base + (int64_t)threadIdx.x;
        const unsigned long long v = i >= 0 ? cmin[i] : ~0ull;
        // inclusive suffix minimum over the threads of this round (Hillis-Steele in LDS)
        buf[threadIdx.x] = v;
        __syncthreads();
        for (uint32_t o = 1; o < 1024; o <<= 1) {
            const unsigned long long y = threadIdx.x + o < 1024 ? buf[threadIdx.x + o] : ~0ull;
            __syncthreads();
            if (y < buf[threadIdx.x]) buf[threadIdx.x] = y;
            __syncthreads();
        }
        const unsigned long long carry = sh_carry;
        const unsigned long long after = threadIdx.x + 1 < 1024 ? buf[threadIdx.x + 1] : ~0ull;
        if (i >= 0) cmin[i] = after < carry ? after : carry;
        __syncthreads();
        if (threadIdx.x == 0) sh_carry = buf[0] < carry ? buf[0] : carry;
        __syncthreads();
    }
}

// Pass 3: out[i] = min(out[i .. end of chunk], cmin[chunk]) -- each chunk's
// suffix minimum from the end, sequential per thread over 16 entries.
__global__ __launch_bounds__(256) void k_min_fill(uint64_t* out, uint64_t n, const uint64_t* cmin)
{
    __shared__ unsigned long long buf[256];
    const uint64_t s = (uint64_t)blockIdx.x * kMinChunk;
    constexpr uint32_t per = kMinChunk / 256;
    const uint64_t p0 = s + (uint64_t)threadIdx.x * per;
    unsigned long long loc[per];
    unsigned long long m = ~0ull;
#pragma unroll
    for (int j = per - 1; j >= 0; --j) {
        const uint64_t i = p0 + j;
        const unsigned long long x = i < n ? out[i] : ~0ull;
        m = x < m ? x : m;
        loc[j] = m;
    }
    // suffix minimum of the threads' minima (thread t needs threads > t)
    buf[threadIdx.x] = m;
    __syncthreads();
    for (uint32_t o = 1; o < 256; o <<= 1) {
        const unsigned long long y = threadIdx.x + o < 256 ? buf[threadIdx.x + o] : ~0ull;
        __syncthreads();
        if (y < buf[threadIdx.x]) buf[threadIdx.x] = y;
        __syncthreads();
    }
    unsigned long long c = threadIdx.x + 1 < 256 ? buf[threadIdx.x + 1] : ~0ull;
    const unsigned long long cc = cmin[blockIdx.x];
    c = cc < c ? cc : c;
#pragma unroll
    for (int j = 0; j < (int)per; ++j) {
        const uint64_t i = p0 + j;
        if (i < n) out[i] = loc[j] < c ? loc[j] : c;
    }
}

// ---------------------------------------------------------------- device-sized levels
// A batch whose level sizes never travel to the host: the first level is
// planned here from the instance offsets, every later level by k_plan_ds, and
// each kernel of a level reads its counts from that level's LevelInfo.

// Zeroes `words` 32-bit words (a kernel, so the call can be captured).
__global__ __launch_bounds__(256) void k_ds_clear(uint32_t* p, uint32_t words)
{
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < words; i += gridDim.x * 256) p[i] = 0;
}

struct JobLists {
    Job* jobs;
    uint64_t base[kJobClasses];
    uint32_t cap[kJobClasses];
};

// Offsets must rise from 0 to n; otherwise no instance is planned at all
// (instances would overlap), and the status says why.
__global__ __launch_bounds__(256) void k_ds_check_offsets(const uint64_t* offs, uint32_t ninst, uint64_t n,
                                                          LevelInfo* info)
{
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < ninst; i += gridDim.x * 256) {
        const uint64_t o0 = offs[i], o1 = offs[i + 1];
        if (o1 < o0 || o1 > n || (i == 0 && o0 != 0) || (i + 1 == ninst && o1 != n))
            atomicOr(&info->status, kStatusBadOffsets);
    }
}

// First level of a batch: instance i is [offs[i], offs[i+1]).  Instances of
// at least alpha records become subproblems, smaller ones base-case jobs by
// capacity class, single records copy jobs (none in place).  The order of the
// lists depends on scheduling; results do not (each entry names its records).
__global__ __launch_bounds__(256) void k_ds_plan_instances(const uint64_t* offs, uint32_t ninst, uint64_t n,
                                                           uint32_t alpha, uint32_t nl0, uint32_t inplace,
                                                           Seg* segs, uint32_t seg_cap, JobLists jl,
                                                           LevelInfo* info)
{
    if (info->status & kStatusBadOffsets) return;  // checked by k_ds_check_offsets
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < ninst; i += gridDim.x * 256) {
        const uint64_t o0 = offs[i], o1 = offs[i + 1];
        const uint32_t len = (uint32_t)(o1 - o0);
        if (len >= alpha) {
            const uint32_t at = atomicAdd(&info->nsegs, 1u);
            if (at < seg_cap) {
                Seg sg;
                sg.start = (uint32_t)o0;
                sg.len = len;
                sg.ibase = (uint32_t)o0;
                sg.tile0 = sg.chunk0 = sg.ntiles = 0;
                const uint32_t nl = choose_nl(len, alpha, kLightBitsMax, 0);
                sg.nl_bits = (uint8_t)(nl < nl0 ? nl : nl0);
                sg.shift = 0;
                sg.nbk = 0;
                sg.nheavy = 0;
                sg.hlog2 = 0;
                segs[at] = sg;
            }
        } else if (len >= 2 || (len == 1 && !inplace)) {
            const int c = len == 1 ? kCopyClass : base_class(len);
            const uint32_t at = atomicAdd(&info->njobs[c], 1u);
            if (at < jl.cap[c]) jl.jobs[jl.base[c] + at] = Job{(uint32_t)o0, len};
        }
    }
}

// After the last device-sized level: folds every level's status into *out,
// and flags subproblems left unfinished or lists that outgrew their room.
__global__ void k_ds_finish(const LevelInfo* infos, uint32_t levels, uint32_t seg_cap, JobLists jl,
                            uint32_t fill_cap, LevelInfo* out)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint32_t st = 0;
    for (uint32_t l = 0; l <= levels; ++l) {
        const LevelInfo& li = infos[l];
        st |= li.status;
        if (li.nsegs > seg_cap) st |= kStatusCapacity;
        for (int c = 0; c < kJobClasses; ++c)
            if (li.njobs[c] > jl.cap[c]) st |= kStatusCapacity;
        if (li.nfills > fill_cap) st |= kStatusCapacity;
    }
    if (infos[levels].nsegs) st |= kStatusTooDeep;
    if (st) atomicOr(&out->status, st);
}

// ================================================================ Step 3
// Local refining base case for semisort_= (Section 3.3).  The paper packs a
// sequential chained hash table in table order.  Here one block per bucket of
// at most CAP = W*512 records, keys and values held in registers:
//   1. keys go to LDS and into an LDS hash table (open addressing; a slot is
//      claimed by CAS and holds the index of a record with that key, keys are
//      compared through that index);
//   2. each record lowers its slot to the smallest index of its key
//      (atomicMin), so f(i) = first occurrence of record i's key, a value
//      that does not depend on scheduling;
//   3. a stable one-pass multisplit on f(i) (ballot match plus per-wave LDS
//      counters) gives every record its output slot: groups in order of first
//      occurrence, input order inside a group (stable).
// Values never touch LDS; results are written straight from registers.

template <int MODE, typename V, int W, typename K = uint64_t>
__device__ __forceinline__ void base_run(const Job* __restrict__ jobs, uint32_t njobs, const K* src_keys,
                                         const V* src_vals, K* out_keys, V* out_vals, uint64_t* sink,
                                         LevelInfo* info)
{
    // Persistent: the grid holds as many blocks as fit on the device, each
    // takes every gridDim.x-th job, and the next job's records are loaded
    // into registers while the current one is refined.  Loads (clamped) and
    // stores (a sink for lanes without a record) are issued unconditionally,
    // so waiting for the prefetched records does not wait for the stores.
    constexpr int BS = W * 64, E = 8, CAP = BS * E;
    __shared__ KReg<K> kl[CAP];
    __shared__ uint32_t tab[2 * CAP];  // slot owners; reused for digit starts
    __shared__ uint16_t wc[W * CAP];
    __shared__ uint32_t tmp[8 * 16 + 8];

    const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    const uint32_t lofs = w * 64 * E + lane;
    K* sink_k = (K*)sink + lane;
    V* sink_v = (V*)(sink + lane);
    uint32_t jb = blockIdx.x;
    if (jb >= njobs) return;
    Job jn = jobs[jb];
    KReg<K> kn[E];
    V vn[E];
    auto fetch = [&](const Job& jj) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t i = min(lofs + e * 64u, jj.len - 1);  // len >= 2
            kn[e] = kload(src_keys + jj.start + i);
            vn[e] = src_vals[jj.start + i];
        }
    };
    fetch(jn);
    bool bad = false;
    for (; jb < njobs; jb += gridDim.x) {
        const Job j = jn;
        KReg<K> k[E];
        V v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            k[e] = kn[e];
            v[e] = vn[e];
        }
        // the next job (the last one re-reads itself); a wave-uniform index
        // makes the descriptor a scalar load, whose wait does not drain the
        // vector memory counter (stores and the prefetch)
        const uint32_t nx = __builtin_amdgcn_readfirstlane(jb + gridDim.x < njobs ? jb + gridDim.x : jb);
        jn = jobs[nx];
        fetch(jn);

        const uint32_t m = j.len;  // 2 .. CAP
        const uint64_t start = j.start;
        const uint32_t lg = ceil_log2_u32(2 * m) < 6 ? 6 : ceil_log2_u32(2 * m);
        const uint32_t slots = 1u << lg, smask = slots - 1;
        const uint32_t nbits = ceil_log2_u32(m);

#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t i = lofs + e * 64u;
            if (i < m) kl[i] = k[e];
        }
        for (uint32_t i = tid; i < slots; i += BS) tab[i] = kEmpty32;
        for (uint32_t i = tid; i < (uint32_t)(W * CAP) / 2; i += BS) ((uint32_t*)wc)[i] = 0;
        __syncthreads();

        // Insertion: a compare-and-swap claims an empty slot or returns its
        // owner in one LDS round trip.  The slot comes from the key itself
        // (Fibonacci hashing of the folded key): a bucket's keys agree only
        // in bits of their mixed hash, not in bits of the key.
        uint32_t sl[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t i = lofs + e * 64u;
            sl[e] = 0;
            if (i < m) {
                uint32_t s = fib_slot(kfold(k[e]), lg);
                while (true) {
                    const uint32_t o = atomicCAS(&tab[s], kEmpty32, i);
                    if (o == kEmpty32 || kl[o] == k[e]) break;
                    s = (s + 1) & smask;
                }
                sl[e] = s;
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t i = lofs + e * 64u;
            if (i < m) atomicMin(&tab[sl[e]], i);
        }
        __syncthreads();
        uint32_t f[E], rk[E];
#pragma unroll
        for (int e = 0; e < E; ++e) f[e] = tab[sl[e]];
        uint16_t* wcw = wc + w * CAP;
        {
            bool ok[E];
#pragma unroll
            for (int e = 0; e < E; ++e) ok[e] = lofs + e * 64u < m;
            wave_rank_all<E, ilog2_c(CAP)>(f, ok, nbits, wcw, rk);
        }
        __syncthreads();
        // per digit: prefix over waves, total; exclusive scan of the totals
        // over the m digits.  Digit d = e*BS + tid belongs to thread tid, so
        // that neighbouring lanes touch neighbouring counters (no bank
        // conflicts).
        uint32_t* dstart = tab;  // the table is no longer needed
        uint32_t tot[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t d = e * BS + tid;
            uint32_t run = 0;
            if (d < m) {
#pragma unroll
                for (int ww = 0; ww < W; ++ww) {
                    const uint32_t c = wc[ww * CAP + d];
                    wc[ww * CAP + d] = (uint16_t)run;
                    run += c;
                }
            }
            tot[e] = run;
        }
        uint32_t ex[E];
        block_excl_scan_rows<BS, E>(tot, ex, tmp);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t d = e * BS + tid;
            if (d < m) dstart[d] = ex[e];
        }
        __syncthreads();
        uint32_t pp[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t i = lofs + e * 64u;
            const uint32_t fe = i < m ? f[e] : 0u;
            const uint32_t p = dstart[fe] + wc[w * CAP + fe] + rk[e];
            bad |= i < m && p >= m;
            pp[e] = (i < m && p < m) ? p : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const bool ok = pp[e] != 0xFFFFFFFFu;
            *(ok ? out_keys + start + pp[e] : sink_k) = knarrow<K>(k[e]);
            *(ok ? out_vals + start + pp[e] : sink_v) = v[e];
        }
        __syncthreads();  // the next job reuses the LDS
    }
    if (bad) atomicOr(&info->status, kStatusBaseIndex);
}

template <int MODE, typename V, int W, typename K = uint64_t>
__global__ __launch_bounds__(W * 64) void k_base(const Job* __restrict__ jobs, uint32_t njobs, const K* src_keys,
                                                 const V* src_vals, K* out_keys, V* out_vals,
                                                 uint64_t* sink, LevelInfo* info)
{
    base_run<MODE, V, W, K>(jobs, njobs, src_keys, src_vals, out_keys, out_vals, sink, info);
}

// Device-counted: the class's job count is read from *count (bounded by cap).
template <int MODE, typename V, int W>
__global__ __launch_bounds__(W * 64) void k_base_ds(const Job* __restrict__ jobs, const uint32_t* count, uint32_t cap,
                                                    const uint64_t* src_keys, const V* src_vals, uint64_t* out_keys,
                                                    V* out_vals, uint64_t* sink, LevelInfo* info)
{
    const uint32_t n = *count < cap ? *count : cap;
    base_run<MODE, V, W>(jobs, n, src_keys, src_vals, out_keys, out_vals, sink, info);
}

// The same base case for buckets of up to 4096 records, with the stable
// multisplit on f(i) done as two 6-bit passes (small per-wave counters) so two
// blocks fit on a CU.  Values are gathered from the source by index after the
// sort (the bucket was just read, so the gather hits in L2); all reads finish
// before the first write, so the output may be the source.
template <int MODE, typename V, typename K = uint64_t>
__device__ __forceinline__ void base_2pass_item(const Job j, const K* src_keys, const V* src_vals,
                                                K* out_keys, V* out_vals, LevelInfo* info)
{
    constexpr int W = 8, BS = 512, E = 8, CAP = 4096;
    __shared__ KReg<K> kl[CAP];
    __shared__ uint32_t tab[2 * CAP];  // slot owners, then the two sort buffers
    __shared__ uint16_t wc[W * 64];
    __shared__ uint32_t dst_[64];
    __shared__ uint32_t tmp[20];

    const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    const uint32_t m = j.len;  // 2 .. CAP
    const uint64_t start = j.start;
    const uint32_t lg = ceil_log2_u32(2 * m) < 6 ? 6 : ceil_log2_u32(2 * m);
    const uint32_t slots = 1u << lg, smask = slots - 1;

    KReg<K> k[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t i = w * 64 * E + e * 64 + lane;
        k[e] = KReg<K>{};
        if (i < m) {
            k[e] = kload(src_keys + start + i);
            kl[i] = k[e];
        }
    }
    for (uint32_t i = tid; i < slots; i += BS) tab[i] = kEmpty32;
    __syncthreads();
    uint32_t sl[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t i = w * 64 * E + e * 64 + lane;
        sl[e] = 0;
        if (i < m) {
            // one compare-and-swap claims the slot or returns its owner;
            // Fibonacci hashing of the folded key (as in k_base)
            uint32_t sx = fib_slot(kfold(k[e]), lg);
            while (true) {
                const uint32_t o = atomicCAS(&tab[sx], kEmpty32, i);
                if (o == kEmpty32 || kl[o] == k[e]) break;
                sx = (sx + 1) & smask;
            }
            sl[e] = sx;
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t i = w * 64 * E + e * 64 + lane;
        if (i < m) atomicMin(&tab[sl[e]], i);
    }
    __syncthreads();
    uint32_t el[E];  // (index << 12) | f
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t i = w * 64 * E + e * 64 + lane;
        el[e] = (i << 12) | (i < m ? tab[sl[e]] : 0u);
    }
    __syncthreads();
    uint32_t* A = tab;
    uint32_t* B = tab + CAP;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        const uint32_t sh = pass ? 6u : 0u;
        for (uint32_t i = tid; i < W * 64; i += BS) wc[i] = 0;
        __syncthreads();
        uint32_t rk[E];
        {
            uint32_t dg[E];
            bool ok[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                dg[e] = (el[e] >> sh) & 63u;
                ok[e] = w * 64 * E + e * 64 + lane < m;
            }
            wave_rank_all<E, 6>(dg, ok, 6, wc + w * 64, rk);
        }
        __syncthreads();
        uint32_t dtot = 0;
        if (tid < 64) {
            for (int ww = 0; ww < W; ++ww) {
                const uint32_t c = wc[ww * 64 + tid];
                wc[ww * 64 + tid] = (uint16_t)dtot;
                dtot += c;
            }
        }
        const uint32_t ds = block_excl_scan<BS>(tid < 64 ? dtot : 0u, tmp, nullptr);
        if (tid < 64) dst_[tid] = ds;
        __syncthreads();
        uint32_t* out = pass ? B : A;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t q = w * 64 * E + e * 64 + lane;
            if (q < m) {
                const uint32_t d = (el[e] >> sh) & 63u;
                out[dst_[d] + wc[w * 64 + d] + rk[e]] = el[e];
            }
        }
        __syncthreads();
        if (pass == 0) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const uint32_t q = w * 64 * E + e * 64 + lane;
                el[e] = q < m ? A[q] : 0u;
            }
        }
    }
    KReg<K> ok[E];
    V ov[E];
    bool bad = false;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t q = tid + e * BS;
        if (q < m) {
            uint32_t i = B[q] >> 12;
            if (i >= m) {
                bad = true;
                i = 0;
            }
            ok[e] = kl[i];
            ov[e] = src_vals[start + i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t q = tid + e * BS;
        if (q < m) {
            out_keys[start + q] = knarrow<K>(ok[e]);
            out_vals[start + q] = ov[e];
        }
    }
    if (bad) atomicOr(&info->status, kStatusBaseIndex);
}

template <int MODE, typename V, typename K = uint64_t>
__global__ __launch_bounds__(512) void k_base_2pass(const Job* jobs, const K* src_keys, const V* src_vals,
                                                    K* out_keys, V* out_vals, LevelInfo* info)
{
    base_2pass_item<MODE, V, K>(jobs[blockIdx.x], src_keys, src_vals, out_keys, out_vals, info);
}

template <int MODE, typename V>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_base_2pass_ds(
    const Job* jobs, const uint32_t* count, uint32_t cap, uint32_t* ctr, const uint64_t* src_keys, const V* src_vals,
    uint64_t* out_keys, V* out_vals, LevelInfo* info)
{
    // Jobs differ in size: blocks take the next one from a counter, asking
    // for it (and loading its descriptor) while the current one runs.  Two
    // blocks per CU, as with one block per job (the register cap keeps the
    // loop's extra state from costing occupancy).
    __shared__ uint32_t sh_i;
    __shared__ Job sh_j;
    const uint32_t n = *count < cap ? *count : cap;
    if (threadIdx.x == 0) {
        const uint32_t i = atomicAdd(ctr, 1u);
        sh_i = i;
        if (i < n) sh_j = jobs[i];
    }
    __syncthreads();
    for (uint32_t i = __builtin_amdgcn_readfirstlane(sh_i); i < n;) {
        // block-uniform: scalar registers, as a descriptor loaded by block index
        const Job j{(uint32_t)__builtin_amdgcn_readfirstlane(sh_j.start),
                    (uint32_t)__builtin_amdgcn_readfirstlane(sh_j.len)};
        uint32_t nx = 0;
        Job jn{0u, 0u};
        __syncthreads();  // every thread has read sh_i and sh_j
        if (threadIdx.x == 0) {
            nx = atomicAdd(ctr, 1u);
            if (nx < n) jn = jobs[nx];
        }
        base_2pass_item<MODE, V>(j, src_keys, src_vals, out_keys, out_vals, info);
        if (threadIdx.x == 0) {
            sh_i = nx;
            sh_j = jn;
        }
        __syncthreads();
        i = __builtin_amdgcn_readfirstlane(sh_i);
    }
}

// Base case of semisort_< (Section 3.3: a stable comparison sort of a small
// bucket).  On the GPU a stable LSD radix sort of the bucket in LDS: keys
// are offset by the bucket's minimum and only the bytes in which they differ
// are sorted, 8 bits per pass, each pass a stable multisplit (ballot match
// plus per-wave counters).  All loads precede all stores, so the output may
// be the source.
template <typename V, int W, typename K = uint64_t>
__global__ __launch_bounds__(W * 64) void k_base_less(const Job* jobs, const K* src_keys, const V* src_vals,
                                                      K* out_keys, V* out_vals)
{
    constexpr int BS = W * 64, E = 8, CAP = BS * E;
    __shared__ uint64_t sk[CAP];
    __shared__ V sv[CAP];
    __shared__ uint16_t wc[W * 256];
    __shared__ uint32_t dst_[256];
    __shared__ uint32_t tmp[20];
    __shared__ unsigned long long sh_min, sh_max;

    const Job j = jobs[blockIdx.x];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    const uint32_t m = j.len;
    const uint64_t start = j.start;
    uint64_t k[E];
    V v[E];
    uint64_t mn = ~0ull, mx = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t q = w * 64 * E + e * 64 + lane;
        k[e] = q < m ? (uint64_t)src_keys[start + q] : 0ull;
        v[e] = q < m ? src_vals[start + q] : (V)0;
        if (q < m) {
            mn = k[e] < mn ? k[e] : mn;
            mx = k[e] > mx ? k[e] : mx;
        }
    }
    if (tid == 0) {
        sh_min = ~0ull;
        sh_max = 0;
    }
    __syncthreads();
    atomicMin(&sh_min, (unsigned long long)mn);
    atomicMax(&sh_max, (unsigned long long)mx);
    __syncthreads();
    const uint64_t kmin = sh_min;
    const uint64_t span = sh_max - kmin;
    const uint32_t bits = span ? 64u - (uint32_t)__clzll(span) : 0u;
    const uint32_t npass = (bits + 7) / 8;
    for (uint32_t pass = 0; pass < npass; ++pass) {
        const uint32_t sh = 8 * pass;
        for (uint32_t i = tid; i < W * 256; i += BS) wc[i] = 0;
        __syncthreads();
        uint32_t rk[E];
        {
            uint32_t dg[E];
            bool ok[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                dg[e] = (uint32_t)((k[e] - kmin) >> sh) & 255u;
                ok[e] = w * 64 * E + e * 64 + lane < m;
            }
            wave_rank_all<E, 8>(dg, ok, 8, wc + w * 256, rk);
        }
        __syncthreads();
        // per digit: exclusive prefix over waves, then an exclusive scan of the
        // 256 digit totals
        if constexpr (BS >= 256) {
            uint32_t dtot = 0;
            if (tid < 256) {
                for (int ww = 0; ww < W; ++ww) {
                    const uint32_t c = wc[ww * 256 + tid];
                    wc[ww * 256 + tid] = (uint16_t)dtot;
                    dtot += c;
                }
            }
            const uint32_t ds = block_excl_scan<BS>(tid < 256 ? dtot : 0u, tmp, nullptr);
            if (tid < 256) dst_[tid] = ds;
        } else {
            // fewer than 256 threads: each thread owns 256/BS digits
            constexpr int PD = 256 / BS;
            uint32_t loc[PD];
            uint32_t sum = 0;
            for (int d = 0; d < PD; ++d) {
                const uint32_t dg = tid * PD + d;
                uint32_t t2 = 0;
                for (int ww = 0; ww < W; ++ww) {
                    const uint32_t c = wc[ww * 256 + dg];
                    wc[ww * 256 + dg] = (uint16_t)t2;
                    t2 += c;
                }
                loc[d] = t2;
                sum += t2;
            }
            uint32_t run = block_excl_scan<BS>(sum, tmp, nullptr);
            for (int d = 0; d < PD; ++d) {
                dst_[tid * PD + d] = run;
                run += loc[d];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t q = w * 64 * E + e * 64 + lane;
            if (q < m) {
                const uint32_t d = (uint32_t)((k[e] - kmin) >> sh) & 255u;
                const uint32_t p = dst_[d] + wc[w * 256 + d] + rk[e];
                sk[p] = k[e];
                sv[p] = v[e];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t q = w * 64 * E + e * 64 + lane;
            if (q < m) {
                k[e] = sk[q];
                v[e] = sv[q];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t q = w * 64 * E + e * 64 + lane;
        if (q < m) {
            out_keys[start + q] = (K)k[e];
            out_vals[start + q] = v[e];
        }
    }
}

// Copy jobs: buckets that are final but sit in T (Section 3.4).
template <typename V, typename K = uint64_t>
__device__ __forceinline__ void copy_item(const Job j, const K* src_keys, const V* src_vals,
                                          K* out_keys, V* out_vals)
{
    const uint64_t st = j.start;
    for (uint32_t i = threadIdx.x; i < j.len; i += 256) {
        out_keys[st + i] = src_keys[st + i];
        out_vals[st + i] = src_vals[st + i];
    }
}

template <typename V, typename K = uint64_t>
__global__ __launch_bounds__(256) void k_copy(const Job* jobs, const K* src_keys, const V* src_vals,
                                              K* out_keys, V* out_vals)
{
    copy_item<V, K>(jobs[blockIdx.x], src_keys, src_vals, out_keys, out_vals);
}

template <typename V>
__global__ __launch_bounds__(256) void k_copy_ds(const Job* jobs, const uint32_t* count, uint32_t cap,
                                                 const uint64_t* src_keys, const V* src_vals, uint64_t* out_keys,
                                                 V* out_vals)
{
    const uint32_t n = *count < cap ? *count : cap;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) copy_item<V>(jobs[i], src_keys, src_vals, out_keys, out_vals);
}

// Key-fill jobs: the keys of a one-key bucket are one value repeated.
// 16-byte stores between a head and a tail of fewer than 16 bytes each
// (keys are aligned to their size).
template <typename K = uint64_t>
__device__ __forceinline__ void fill_item(const FillJob j, K* out_keys)
{
    constexpr uint32_t P = 16 / sizeof(K);  // keys per 16-byte store
    K* o = out_keys + j.start;
    const K key = (K)j.key;
    const uint32_t mis = (uint32_t)(((uintptr_t)o & 15u) / sizeof(K));
    const uint32_t head = mis ? (P - mis < j.len ? P - mis : j.len) : 0u;
    const uint32_t n4 = (j.len - head) / P;
    const uint32_t tail = head + n4 * P;
    if (threadIdx.x < head) o[threadIdx.x] = key;
    if (threadIdx.x < j.len - tail) o[tail + threadIdx.x] = key;
    const uint32_t lo = (uint32_t)(uint64_t)key;
    const uint32_t hi = sizeof(K) == 8 ? (uint32_t)((uint64_t)key >> 32) : lo;
    const uint4 kk = make_uint4(lo, hi, lo, hi);
    uint4* o4 = (uint4*)(o + head);
    for (uint32_t i = threadIdx.x; i < n4; i += 1024) o4[i] = kk;
}

template <typename K = uint64_t>
__global__ __launch_bounds__(1024) void k_fill(const FillJob* jobs, K* out_keys)
{
    fill_item<K>(jobs[blockIdx.x], out_keys);
}

// Device-counted: the level's fill-job count is read from *count (bounded by cap).
__global__ __launch_bounds__(1024) void k_fill_ds(const FillJob* jobs, const uint32_t* count, uint32_t cap,
                                                  uint64_t* out_keys)
{
    const uint32_t n = *count < cap ? *count : cap;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) fill_item(jobs[i], out_keys);
}

// Offsets and heavy list of a single-subproblem level, for inspection.
__global__ void k_export_partition(const uint32_t* bstart, const Seg* segs, const uint64_t* heavy_list,
                                   uint64_t* offsets_out, uint64_t* heavy_out)
{
    const Seg sg = segs[0];
    const uint32_t nb = sg.nbk;
    for (uint32_t b = threadIdx.x; b <= nb; b += blockDim.x) offsets_out[b] = bstart[b] - sg.start;
    for (uint32_t h = threadIdx.x; h < sg.nheavy; h += blockDim.x) heavy_out[h] = heavy_list[h];
}

// ================================================================ Section 3.5
// Collect-reduce and histogram on the semisort_= skeleton.  A heavy key needs
// no further work once it is known: its records are summed while the level
// is distributed (they never move) and the sum lands in the one slot its
// bucket reserved.  Light buckets recurse as in the semisort; buckets of one
// record or one key are summed directly, small buckets are reduced in LDS.
// Every result sits at a position inside its bucket's range, marked in rflag;
// a final compaction packs them.  The monoid is wrapping 64-bit addition;
// for the histogram every value is 1.

// Results of the heavy keys of every subproblem of the level.
template <int MODE>
__global__ __launch_bounds__(256) void k_heavy_results(LevelArgs a)
{
    const uint32_t sid = blockIdx.x;
    const Seg sg = a.segs[sid];
    const uint32_t nL = 1u << sg.nl_bits;
    const uint32_t* bs = a.bstart + (size_t)sid * (kNbStride + 1);
    bool bad = false;
    for (uint32_t h = threadIdx.x; h < sg.nheavy; h += 256) {
        const uint32_t b = nL + h;
        const uint32_t p = bs[b];
        if (bs[b + 1] - p != 1u || p - sg.start >= sg.len) {
            bad = true;
            continue;
        }
        a.res_keys[p] = key_of_hash<MODE>(a.heavy_list[(size_t)sid * kHeavyMax + h]);
        a.res_vals[p] = a.hsum[(size_t)sid * kHeavyMax + h];
        a.rflag[p] = 1;
    }
    if (bad) atomicOr(&a.info->status, kStatusSizeMismatch);
}

// First / last value per key (non-commutative monoids, exact through a stable
// order): the record positions are reduced with min / max, then each result
// position is replaced by the value at it.
__global__ __launch_bounds__(256) void k_iota(uint64_t* p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) p[i] = i;
}

__global__ __launch_bounds__(256) void k_gather_at(uint64_t* out, uint64_t m, const uint64_t* vals, uint64_t n,
                                                   LevelInfo* info)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (uint64_t)gridDim.x * 256) {
        const uint64_t p = out[i];
        if (p >= n) {
            atomicOr(&info->status, kStatusSizeMismatch);
            continue;
        }
        out[i] = vals[p];
    }
}

// The same with m read from device memory (m <= n; the grid covers n).
__global__ __launch_bounds__(256) void k_gather_at_dev(uint64_t* out, const uint64_t* m, const uint64_t* vals,
                                                       uint64_t n, LevelInfo* info)
{
    const uint64_t mm = *m;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < mm; i += (uint64_t)gridDim.x * 256) {
        const uint64_t p = out[i];
        if (p >= n) {
            atomicOr(&info->status, kStatusSizeMismatch);
            continue;
        }
        out[i] = vals[p];
    }
}

// ---------------------------------------------------------------- in-order folds
// Section 3.5: a stable algorithm reduces with any associative operation,
// commutative or not.  After a stable semisort_= each key's records are
// contiguous and in input order, so a segmented scan in position order folds
// every group.  The operation here composes affine maps on 32-bit integers:
// a value holds (a, b) = (high, low 32 bits) for t -> a t + b mod 2^32, and
// x then y = (a_y a_x, a_y b_x + b_y) mod 2^32, identity (1, 0).

constexpr uint64_t kAffineId = 1ull << 32;
constexpr uint32_t kFoldChunk = 4096;  // positions per block (256 threads x 16)

__device__ __forceinline__ uint64_t affine_then(uint64_t x, uint64_t y)
{
    const uint32_t ax = (uint32_t)(x >> 32), bx = (uint32_t)x;
    const uint32_t ay = (uint32_t)(y >> 32), by = (uint32_t)y;
    return ((uint64_t)(ay * ax) << 32) | (uint32_t)(ay * bx + by);
}

// Segmented pairs (fold, a group starts inside): (v, f) then (w, g) is
// (g ? w : v then w, f or g); associative because the fold is.
struct SegPair {
    uint64_t v;
    uint32_t f;
};

__device__ __forceinline__ SegPair seg_then(SegPair l, SegPair r)
{
    return SegPair{r.f ? r.v : affine_then(l.v, r.v), l.f | r.f};
}

// Block-wide inclusive scan of one pair per thread, in thread order.
__device__ __forceinline__ SegPair seg_block_scan(SegPair x, uint64_t* bv, uint32_t* bf)
{
    const uint32_t t = threadIdx.x;
    bv[t] = x.v;
    bf[t] = x.f;
    __syncthreads();
    for (uint32_t o = 1; o < 256; o <<= 1) {
        SegPair y = x;
        if (t >= o) y = seg_then(SegPair{bv[t - o], bf[t - o]}, x);
        __syncthreads();
        bv[t] = y.v;
        bf[t] = y.f;
        x = y;
        __syncthreads();
    }
    return x;
}

// A chunk of grouped records staged in LDS with coalesced loads; thread t's
// 16 consecutive positions sit at t * 17 .. t * 17 + 15 (one slot of padding
// per thread keeps the per-thread walks off shared banks).  Also the keys
// just before and just after the chunk (for the group boundaries).
constexpr uint32_t kFoldPer = kFoldChunk / 256;
constexpr uint32_t kFoldSlots = 256 * (kFoldPer + 1);

__device__ __forceinline__ void stage_chunk(const uint64_t* sk, const uint64_t* sv, uint64_t n, uint64_t base,
                                            uint64_t* lk, uint64_t* lv, uint64_t* prev_next)
{
    // every load of the chunk in flight before the first LDS store (coalesced:
    // thread t reads positions t, t + 256, ...)
    uint64_t kr[kFoldPer], vr[kFoldPer];
#pragma unroll
    for (uint32_t u = 0; u < kFoldPer; ++u) {
        const uint64_t i = base + u * 256 + threadIdx.x;
        kr[u] = i < n ? sk[i] : 0ull;
        vr[u] = i < n ? sv[i] : 0ull;
    }
#pragma unroll
    for (uint32_t u = 0; u < kFoldPer; ++u) {
        const uint32_t j = u * 256 + threadIdx.x;
        const uint32_t slot = (j / kFoldPer) * (kFoldPer + 1) + j % kFoldPer;
        lk[slot] = kr[u];
        lv[slot] = vr[u];
    }
    if (threadIdx.x == 0) prev_next[0] = base ? sk[base - 1] : 0ull;
    if (threadIdx.x == 1) prev_next[1] = base + kFoldChunk < n ? sk[base + kFoldChunk] : 0ull;
    __syncthreads();
}

// Key of in-chunk position j from the staged chunk (j = -1 and kFoldChunk
// give the neighbours).
__device__ __forceinline__ uint64_t staged_key(const uint64_t* lk, const uint64_t* prev_next, int32_t j)
{
    if (j < 0) return prev_next[0];
    if (j >= (int32_t)kFoldChunk) return prev_next[1];
    return lk[(j / kFoldPer) * (kFoldPer + 1) + j % kFoldPer];
}

__device__ __forceinline__ SegPair fold_thread_range(const uint64_t* lk, const uint64_t* lv, const uint64_t* pn,
                                                     uint64_t n, uint64_t base)
{
    SegPair acc{kAffineId, 0u};
    const uint32_t t = threadIdx.x;
    for (uint32_t j = 0; j < kFoldPer; ++j) {
        const uint32_t q = t * kFoldPer + j;
        if (base + q >= n) break;
        const uint64_t k = lk[t * (kFoldPer + 1) + j];
        const uint32_t st = base + q == 0 || k != staged_key(lk, pn, (int32_t)q - 1);
        acc = seg_then(acc, SegPair{lv[t * (kFoldPer + 1) + j], st});
    }
    return acc;
}

// Pass 1: the segmented fold of every chunk of positions.
__global__ __launch_bounds__(256) void k_sfold_aggr(const uint64_t* sk, const uint64_t* sv, uint64_t n,
                                                    uint64_t* aggv, uint32_t* aggf)
{
    __shared__ uint64_t lk[kFoldSlots];
    __shared__ uint64_t lv[kFoldSlots];
    __shared__ uint64_t pn[2];
    __shared__ uint64_t bv[256];
    __shared__ uint32_t bf[256];
    const uint64_t base = (uint64_t)blockIdx.x * kFoldChunk;
    stage_chunk(sk, sv, n, base, lk, lv, pn);
    const SegPair x = seg_block_scan(fold_thread_range(lk, lv, pn, n, base), bv, bf);
    if (threadIdx.x == 255) {
        aggv[blockIdx.x] = x.v;
        aggf[blockIdx.x] = x.f;
    }
}

// Pass 2, in two levels.  2a: each block scans 256 chunk folds in place
// (exclusive, flags kept) and writes their total; 2b (one block of 1024):
// the block totals become exclusive carries.  The fold open at the start of
// chunk c is then carry[c / 256] then the in-block prefix of c.
__global__ __launch_bounds__(256) void k_sfold_carry_blocks(uint64_t* aggv, uint32_t* aggf, uint32_t nch,
                                                            uint64_t* totv, uint32_t* totf)
{
    __shared__ uint64_t bv[256];
    __shared__ uint32_t bf[256];
    const uint32_t c = blockIdx.x * 256 + threadIdx.x;
    const SegPair mine = c < nch ? SegPair{aggv[c], aggf[c]} : SegPair{kAffineId, 0u};
    const SegPair inc = seg_block_scan(mine, bv, bf);
    const SegPair excl = threadIdx.x ? SegPair{bv[threadIdx.x - 1], bf[threadIdx.x - 1]} : SegPair{kAffineId, 0u};
    if (c < nch) {
        aggv[c] = excl.v;
        aggf[c] = excl.f;
    }
    if (threadIdx.x == 255) {
        totv[blockIdx.x] = inc.v;
        totf[blockIdx.x] = inc.f;
    }
}

__global__ __launch_bounds__(1024) void k_sfold_carry_top(uint64_t* totv, uint32_t* totf, uint32_t nb, uint32_t rb)
{
    // rounds of rb <= 1024 block totals (a power of two), Hillis-Steele in
    // LDS; the fold of every earlier round is carried into the next
    __shared__ uint64_t bv[1024];
    __shared__ uint32_t bf[1024];
    __shared__ uint64_t sh_cv;
    __shared__ uint32_t sh_cf;
    const uint32_t t = threadIdx.x;
    if (t == 0) {
        sh_cv = kAffineId;
        sh_cf = 0;
    }
    __syncthreads();
    for (uint32_t base = 0; base < nb; base += rb) {
        const uint32_t i = base + t;
        const bool mine = t < rb && i < nb;
        SegPair x = mine ? SegPair{totv[i], totf[i]} : SegPair{kAffineId, 0u};
        bv[t] = x.v;
        bf[t] = x.f;
        __syncthreads();
        for (uint32_t o = 1; o < 1024; o <<= 1) {
            SegPair y = x;
            if (t >= o) y = seg_then(SegPair{bv[t - o], bf[t - o]}, x);
            __syncthreads();
            bv[t] = y.v;
            bf[t] = y.f;
            x = y;
            __syncthreads();
        }
        const SegPair carry{sh_cv, sh_cf};
        const SegPair before = t ? seg_then(carry, SegPair{bv[t - 1], bf[t - 1]}) : carry;
        __syncthreads();
        if (mine) {
            totv[i] = before.v;
            totf[i] = before.f;
        }
        if (t == rb - 1) {
            const SegPair next = seg_then(carry, x);
            sh_cv = next.v;
            sh_cf = next.f;
        }
        __syncthreads();
    }
}

// Pass 3: each group's fold, written at its last position (the position
// order of the flagged results is the group order of the semisort).
__global__ __launch_bounds__(256) void k_sfold_apply(const uint64_t* sk, const uint64_t* sv, uint64_t n,
                                                     const uint64_t* aggv, const uint32_t* aggf, const uint64_t* totv,
                                                     uint64_t* res_keys, uint64_t* res_vals, uint8_t* rflag)
{
    __shared__ uint64_t lk[kFoldSlots];
    __shared__ uint64_t lv[kFoldSlots];
    __shared__ uint64_t pn[2];
    __shared__ uint64_t bv[256];
    __shared__ uint32_t bf[256];
    const uint64_t base = (uint64_t)blockIdx.x * kFoldChunk;
    stage_chunk(sk, sv, n, base, lk, lv, pn);
    seg_block_scan(fold_thread_range(lk, lv, pn, n, base), bv, bf);
    // the fold open at this chunk's start: its block's carry, then the
    // chunks before it in that block
    const SegPair chunk_in = seg_then(SegPair{totv[blockIdx.x / 256], 0u}, SegPair{aggv[blockIdx.x], aggf[blockIdx.x]});
    const uint32_t t = threadIdx.x;
    SegPair acc = t ? seg_then(chunk_in, SegPair{bv[t - 1], bf[t - 1]}) : chunk_in;
    for (uint32_t j = 0; j < kFoldPer; ++j) {
        const uint32_t q = t * kFoldPer + j;
        const uint64_t i = base + q;
        if (i >= n) break;
        const uint64_t k = lk[t * (kFoldPer + 1) + j];
        const uint32_t st = i == 0 || k != staged_key(lk, pn, (int32_t)q - 1);
        acc = seg_then(acc, SegPair{lv[t * (kFoldPer + 1) + j], st});
        if (i + 1 == n || staged_key(lk, pn, (int32_t)q + 1) != k) {
            res_keys[i] = k;
            res_vals[i] = acc.v;
            rflag[i] = 1;
        }
    }
}

// Sum jobs: a bucket whose records all share one key, folded with the
// monoid op.  One block per job; all reads finish (block reduction) before
// the single write.
template <int ONES>
__global__ __launch_bounds__(256) void k_sum_job(const Job* jobs, const uint64_t* src_keys, const uint64_t* src_vals,
                                                 uint64_t* res_keys, uint64_t* res_vals, uint8_t* rflag, uint32_t op)
{
    __shared__ unsigned long long acc;
    const Job j = jobs[blockIdx.x];
    const unsigned long long id = red_identity(op);
    if (threadIdx.x == 0) acc = id;
    __syncthreads();
    unsigned long long s = id;
    if constexpr (ONES) {
        s = threadIdx.x == 0 ? j.len : 0u;
    } else {
        for (uint32_t i = threadIdx.x; i < j.len; i += 256) s = red_combine(op, s, src_vals[(uint64_t)j.start + i]);
    }
    const uint64_t k = src_keys[j.start];
    if (s != id) red_atomic(op, &acc, s);
    __syncthreads();
    if (threadIdx.x == 0) {
        res_keys[j.start] = k;
        res_vals[j.start] = acc;
        rflag[j.start] = 1;
    }
}

// Base case of collect-reduce for a bucket of at most CAP = W*512 records:
// an LDS hash table (slot claimed by CAS, keys compared through the owner's
// index) folds each key's values with LDS atomics of the monoid and the smallest index
// of the key, f; the record at f writes (key, sum) at start + f.  Positions
// and sums do not depend on scheduling.  All reads precede all writes, so
// the results may go to the source array.
template <int MODE, int W, int ONES>
__global__ __launch_bounds__(W * 64) void k_base_red(const Job* jobs, const uint64_t* src_keys,
                                                     const uint64_t* src_vals, uint64_t* res_keys,
                                                     uint64_t* res_vals, uint8_t* rflag, uint32_t op)
{
    constexpr int BS = W * 64, E = 8, CAP = BS * E;
    __shared__ uint64_t kl[CAP];
    __shared__ uint32_t tab[2 * CAP];
    __shared__ unsigned long long ssum[2 * CAP];

    const Job j = jobs[blockIdx.x];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    const uint32_t m = j.len;  // 2 .. CAP
    const uint64_t start = j.start;
    const uint32_t lg = ceil_log2_u32(2 * m) < 6 ? 6 : ceil_log2_u32(2 * m);
    const uint32_t slots = 1u << lg, smask = slots - 1;

    uint64_t k[E], v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t i = w * 64 * E + e * 64 + lane;
        k[e] = i < m ? src_keys[start + i] : 0ull;
        if constexpr (ONES) v[e] = 1;
        else v[e] = i < m ? src_vals[start + i] : 0ull;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t i = w * 64 * E + e * 64 + lane;
        if (i < m) kl[i] = k[e];
    }
    for (uint32_t i = tid; i < slots; i += BS) {
        tab[i] = kEmpty32;
        ssum[i] = red_identity(op);
    }
    __syncthreads();
    uint32_t sl[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t i = w * 64 * E + e * 64 + lane;
        sl[e] = 0;
        if (i < m) {
            // one compare-and-swap claims the slot or returns its owner;
            // Fibonacci hashing of the folded key (as in k_base)
            uint32_t sidx = fib_slot(k[e], lg);
            while (true) {
                const uint32_t o = atomicCAS(&tab[sidx], kEmpty32, i);
                if (o == kEmpty32 || kl[o] == k[e]) break;
                sidx = (sidx + 1) & smask;
            }
            sl[e] = sidx;
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t i = w * 64 * E + e * 64 + lane;
        if (i < m) {
            atomicMin(&tab[sl[e]], i);
            red_atomic(op, &ssum[sl[e]], (unsigned long long)v[e]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t i = w * 64 * E + e * 64 + lane;
        if (i < m && tab[sl[e]] == i) {
            res_keys[start + i] = k[e];
            res_vals[start + i] = ssum[sl[e]];
            rflag[start + i] = 1;
        }
    }
}

// Compaction of the results.  Positions are cut into chunks of kFlagChunk,
// one per wave (16 per block of kFlagBlock); a wave walks its chunk in rounds
// of 256 positions, each lane owning 4 neighbouring flag bytes, so flag and
// result reads and the packed writes are coalesced.  Flags are 0 or 1; the
// flag array is padded to a whole number of blocks and cleared before the run.
constexpr uint32_t kFlagBlock = 65536;
constexpr uint32_t kFlagChunk = 4096;

__device__ __forceinline__ uint32_t wave_excl_sum(uint32_t v, uint32_t* total)
{
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    *total = __shfl(x, 63, 64);
    return x - v;
}

// Results per chunk (one wave per chunk), and per block of 16 chunks.
__global__ __launch_bounds__(1024) void k_flag_count(const uint8_t* rflag, uint32_t* ccnt, uint32_t* btot)
{
    __shared__ uint32_t wt[16];
    const uint32_t w = threadIdx.x >> 6;
    const uint32_t chunk = blockIdx.x * 16 + w;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t* f = (const uint64_t*)(rflag + (size_t)chunk * kFlagChunk) + lane * 8;
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) c += __popcll(f[q]);
    uint32_t tot = 0;
    (void)wave_excl_sum(c, &tot);
    if (lane == 0) {
        ccnt[chunk] = tot;
        wt[w] = tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) t += wt[q];
        btot[blockIdx.x] = t;
    }
}

// Exclusive scan of the block totals in place (one block, contiguous runs per
// thread); m to *m_out.
__global__ __launch_bounds__(1024) void k_flag_scan(uint32_t* btot, uint32_t nblk, unsigned long long* m_out)
{
    __shared__ uint32_t tmp[20];
    const uint32_t per = (nblk + 1023) / 1024;
    const uint32_t c0 = threadIdx.x * per;
    const uint32_t c1 = c0 + per < nblk ? c0 + per : nblk;
    uint32_t s = 0;
    for (uint32_t c = c0; c < c1; ++c) s += btot[c];
    uint32_t tot = 0;
    uint32_t run = block_excl_scan<1024>(s, tmp, &tot);
    for (uint32_t c = c0; c < c1; ++c) {
        const uint32_t x = btot[c];
        btot[c] = run;
        run += x;
    }
    if (threadIdx.x == 0) *m_out = tot;
}

// One wave per chunk; its offset is the block's (scanned) plus the counts of
// the block's earlier chunks.  Four rounds of 256 positions at a time, each
// lane owning 4 neighbouring positions: where a group holds at least 1/8
// results, keys and values of all its positions are read with 16-byte loads
// issued together (whole lines, no dependent gathers); sparser groups (and
// the groups at the end of the array) gather only the flagged positions.
__global__ __launch_bounds__(1024) void k_flag_scatter(const uint8_t* rflag, const uint32_t* ccnt,
                                                       const uint32_t* boff, uint64_t n,
                                                       const uint64_t* res_keys, const uint64_t* res_vals,
                                                       uint64_t* out_keys, uint64_t* out_vals)
{
    constexpr int R = 4;
    __shared__ uint32_t sc[16];
    const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t chunk = blockIdx.x * 16 + w;
    if (threadIdx.x < 16) sc[threadIdx.x] = ccnt[blockIdx.x * 16 + threadIdx.x];
    __syncthreads();
    uint32_t o = boff[blockIdx.x];
    for (uint32_t q = 0; q < w; ++q) o += sc[q];
    if (sc[w] == 0) return;
    const size_t base = (size_t)chunk * kFlagChunk;
    for (uint32_t r0 = 0; r0 < kFlagChunk / 256; r0 += R) {
        uint32_t f[R], at[R];
        uint32_t gsum = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            f[r] = *(const uint32_t*)(rflag + base + (r0 + r) * 256 + lane * 4);
            uint32_t tot = 0;
            at[r] = o + wave_excl_sum(__popc(f[r]), &tot);
            o += tot;
            gsum += tot;
        }
        if (gsum == 0) continue;
        const size_t g0 = base + r0 * 256;
        if (gsum >= R * 32 && g0 + R * 256 <= n) {
            ulonglong2 ka[R], kb[R], va[R], vb[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const size_t p = g0 + r * 256 + lane * 4;
                ka[r] = *(const ulonglong2*)(res_keys + p);
                kb[r] = *(const ulonglong2*)(res_keys + p + 2);
                va[r] = *(const ulonglong2*)(res_vals + p);
                vb[r] = *(const ulonglong2*)(res_vals + p + 2);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint64_t kx[4] = {ka[r].x, ka[r].y, kb[r].x, kb[r].y};
                const uint64_t vx[4] = {va[r].x, va[r].y, vb[r].x, vb[r].y};
                uint32_t a = at[r];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    if ((f[r] >> (8 * b)) & 1u) {
                        out_keys[a] = kx[b];
                        out_vals[a] = vx[b];
                        ++a;
                    }
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const size_t p = g0 + r * 256 + lane * 4;
                uint32_t a = at[r];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    if ((f[r] >> (8 * b)) & 1u) {
                        out_keys[a] = res_keys[p + b];
                        out_vals[a] = res_vals[p + b];
                        ++a;
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- batches of jobs
// A batch packs small jobs back to back: job j occupies [off, off + n) of
// the packed arrays.  Gathering and scattering walk the packed array in
// chunks; a chunk finds its first job by binary search over the offsets.

struct PackJob {
    const uint64_t* keys;
    const void* vals;
    void* out_a;
    void* out_b;
    uint64_t* d_m;
    uint64_t off;
    uint64_t n;
};

constexpr uint32_t kPackChunk = 4096;  // packed positions per block

// Largest j < njobs with at[j] <= x (at[] non-decreasing, at[0] <= x).
__device__ __forceinline__ uint32_t last_at_or_below(const uint64_t* at, size_t stride, uint32_t njobs, uint64_t x)
{
    uint32_t lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (at[(size_t)mid * stride] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Inputs of the packed jobs into the packed arrays (pv NULL: keys only).
template <typename V>
__global__ __launch_bounds__(256) void k_pack_gather(const PackJob* jobs, uint32_t njobs, uint64_t total,
                                                     uint64_t* pk, V* pv)
{
    __shared__ uint32_t sj;
    const uint64_t r0 = (uint64_t)blockIdx.x * kPackChunk;
    if (r0 >= total) return;
    const uint64_t r1 = r0 + kPackChunk < total ? r0 + kPackChunk : total;
    if (threadIdx.x == 0) sj = last_at_or_below(&jobs[0].off, sizeof(PackJob) / 8, njobs, r0);
    __syncthreads();
    for (uint32_t j = sj; j < njobs && jobs[j].off < r1; ++j) {
        const PackJob J = jobs[j];
        const uint64_t a = r0 > J.off ? r0 : J.off;
        const uint64_t b = r1 < J.off + J.n ? r1 : J.off + J.n;
        for (uint64_t i = a + threadIdx.x; i < b; i += 256) {
            pk[i] = J.keys[i - J.off];
            if (pv) pv[i] = ((const V*)J.vals)[i - J.off];
        }
    }
}

// Packed semisort results back to every job's outputs.
template <typename V>
__global__ __launch_bounds__(256) void k_pack_scatter(const PackJob* jobs, uint32_t njobs, uint64_t total,
                                                      const uint64_t* ok, const V* ov)
{
    __shared__ uint32_t sj;
    const uint64_t r0 = (uint64_t)blockIdx.x * kPackChunk;
    if (r0 >= total) return;
    const uint64_t r1 = r0 + kPackChunk < total ? r0 + kPackChunk : total;
    if (threadIdx.x == 0) sj = last_at_or_below(&jobs[0].off, sizeof(PackJob) / 8, njobs, r0);
    __syncthreads();
    for (uint32_t j = sj; j < njobs && jobs[j].off < r1; ++j) {
        const PackJob J = jobs[j];
        const uint64_t a = r0 > J.off ? r0 : J.off;
        const uint64_t b = r1 < J.off + J.n ? r1 : J.off + J.n;
        for (uint64_t i = a + threadIdx.x; i < b; i += 256) {
            ((uint64_t*)J.out_a)[i - J.off] = ok[i];
            ((V*)J.out_b)[i - J.off] = ov[i];
        }
    }
}

// Rank among all packed results of the first result of job j (j = njobs:
// the total m): the results are packed in position order, so the rank is the
// number of flagged positions below the job's offset -- its flag block's
// scanned total, the counts of the block's earlier chunks and the flags of
// its own chunk below it.  One block per boundary.
__global__ __launch_bounds__(256) void k_inst_ranks(const uint8_t* rflag, const uint32_t* ccnt, const uint32_t* boff,
                                                    const PackJob* jobs, uint32_t njobs,
                                                    const unsigned long long* m_total, uint64_t* rank)
{
    __shared__ uint32_t ws[4];
    const uint32_t j = blockIdx.x;
    if (j == njobs) {
        if (threadIdx.x == 0) rank[j] = *m_total;
        return;
    }
    const uint64_t x = jobs[j].off;
    const uint64_t blk = x / kFlagBlock, ch = x / kFlagChunk;
    uint32_t c = 0;
    for (uint64_t q = blk * (kFlagBlock / kFlagChunk) + threadIdx.x; q < ch; q += 256) c += ccnt[q];
    for (uint64_t i = ch * kFlagChunk + threadIdx.x; i < x; i += 256) c += rflag[i] != 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if ((threadIdx.x & 63u) == 0) ws[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) rank[j] = (uint64_t)boff[blk] + ws[0] + ws[1] + ws[2] + ws[3];
}

// m of every job to its d_m.
__global__ __launch_bounds__(256) void k_inst_m(const PackJob* jobs, uint32_t njobs, const uint64_t* rank)
{
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j < njobs) *jobs[j].d_m = rank[j + 1] - rank[j];
}

// Packed (key, result) pairs back to every job's outputs: positions
// [rank[j], rank[j + 1]) of the packed pairs are job j's.
__global__ __launch_bounds__(256) void k_pack_scatter_red(const PackJob* jobs, uint32_t njobs, const uint64_t* rank,
                                                          const uint64_t* ok, const uint64_t* ov)
{
    __shared__ uint32_t sj;
    const uint64_t m = rank[njobs];
    const uint64_t r0 = (uint64_t)blockIdx.x * kPackChunk;
    if (r0 >= m) return;
    const uint64_t r1 = r0 + kPackChunk < m ? r0 + kPackChunk : m;
    if (threadIdx.x == 0) sj = last_at_or_below(rank, 1, njobs, r0);
    __syncthreads();
    for (uint32_t j = sj; j < njobs && rank[j] < r1; ++j) {
        const PackJob J = jobs[j];
        const uint64_t s = rank[j], e = rank[j + 1];
        const uint64_t a = r0 > s ? r0 : s;
        const uint64_t b = r1 < e ? r1 : e;
        for (uint64_t i = a + threadIdx.x; i < b; i += 256) {
            ((uint64_t*)J.out_a)[i - s] = ok[i];
            ((uint64_t*)J.out_b)[i - s] = ov[i];
        }
    }
}


// ================================================================ semisort_< of 128-bit keys
// After a stable semisort_= the records of a key form one run, in input
// order.  These kernels number the runs, list each run's start and key words,
// and, once the runs are sorted by key, move every record to its run's place
// in that order: groups in ascending key order, records of a key in input
// order (Section 2.1's semisort_<, stable as in Section 2.2).

constexpr uint32_t kRunChunk = 4096;              // positions per block
constexpr uint32_t kRunPer = kRunChunk / 256;     // positions per thread
constexpr uint32_t kRunWords = kRunChunk / 32;    // words of the chunk's run-start bitmap

// Run starts of a chunk into an LDS bitmap (bit i: a run starts at the
// chunk's position i) and the popcount prefix of its words; thread t looks at
// positions t, t + 256, ... (coalesced loads) and keeps their keys.  Returns
// the chunk's run count.
__device__ __forceinline__ uint32_t run_bitmap(const Key128* k, uint64_t n, uint64_t base, uint32_t* bm,
                                               uint32_t* wpre, uint32_t* tmp, Key128 (&kk)[kRunPer])
{
    const uint32_t t = threadIdx.x;
    for (uint32_t w = t; w < kRunWords; w += 256) bm[w] = 0;
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kRunPer; ++j) {
        const uint64_t i = base + j * 256 + t;
        if (i < n) {
            kk[j] = k[i];
            if (i == 0 || !(kk[j] == k[i - 1])) atomicOr(&bm[(j * 256 + t) >> 5], 1u << (t & 31u));
        }
    }
    __syncthreads();
    const uint32_t c = t < kRunWords ? (uint32_t)__popc(bm[t]) : 0u;
    uint32_t tot = 0;
    const uint32_t ex = block_excl_scan<256>(c, tmp, &tot);
    if (t < kRunWords) wpre[t] = ex;
    __syncthreads();
    return tot;
}

// Runs starting in each chunk of positions, and the chunk's run-start bitmap
// (kRunWords words per chunk) for the passes after it.
__global__ __launch_bounds__(256) void k_runs_count(const Key128* k, uint64_t n, uint32_t* cnt, uint32_t* bits)
{
    __shared__ uint32_t bm[kRunWords], wpre[kRunWords], tmp[20];
    Key128 kk[kRunPer];
    const uint32_t tot = run_bitmap(k, n, (uint64_t)blockIdx.x * kRunChunk, bm, wpre, tmp, kk);
    if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
    for (uint32_t w = threadIdx.x; w < kRunWords; w += 256) bits[(size_t)blockIdx.x * kRunWords + w] = bm[w];
}

// A chunk's stored run-start bitmap into LDS, with the popcount prefix of its
// words (as run_bitmap leaves them).
__device__ __forceinline__ void load_run_bitmap(const uint32_t* bits, uint32_t* bm, uint32_t* wpre, uint32_t* tmp)
{
    const uint32_t t = threadIdx.x;
    const uint32_t w = t < kRunWords ? bits[(size_t)blockIdx.x * kRunWords + t] : 0u;
    if (t < kRunWords) bm[t] = w;
    const uint32_t ex = block_excl_scan<256>((uint32_t)__popc(w), tmp, nullptr);
    if (t < kRunWords) wpre[t] = ex;
    __syncthreads();
}

// In place: exclusive prefix of v[0, count) (one block, rounds of 1024 with
// the earlier rounds' sum carried in); the total to *total.
__global__ __launch_bounds__(1024) void k_scan_u32(uint32_t* v, uint32_t count, uint32_t* total)
{
    __shared__ uint32_t tmp[20];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t b = 0; b < count; b += 1024) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t x = i < count ? v[i] : 0u;
        uint32_t tot = 0;
        const uint32_t ex = block_excl_scan<1024>(x, tmp, &tot);
        const uint32_t c0 = carry;
        if (i < count) v[i] = c0 + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = c0 + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// Run number of chunk position q: the run starts at positions <= q of the
// chunk plus the runs before it (cbase), minus one (position 0 starts run 0).
__device__ __forceinline__ uint32_t run_of(const uint32_t* bm, const uint32_t* wpre, uint32_t c0, uint32_t q)
{
    const uint32_t word = bm[q >> 5], bit = q & 31u;
    return c0 + wpre[q >> 5] + (uint32_t)__popc(word & (0xFFFFFFFFu >> (31u - bit))) - 1u;
}

// Per run: its start and its key's words, from the stored run-start bitmap
// (only the keys at run starts are read).  cbase: runs before each chunk.
__global__ __launch_bounds__(256) void k_runs_emit(const Key128* k, uint64_t n, const uint32_t* cbase,
                                                    const uint32_t* bits, uint32_t* gstart, uint64_t* glo,
                                                    uint64_t* ghi)
{
    __shared__ uint32_t bm[kRunWords], wpre[kRunWords], tmp[20];
    load_run_bitmap(bits, bm, wpre, tmp);
    const uint64_t base = (uint64_t)blockIdx.x * kRunChunk;
    const uint32_t t = threadIdx.x, c0 = cbase[blockIdx.x];
#pragma unroll
    for (uint32_t j = 0; j < kRunPer; ++j) {
        const uint32_t q = j * 256 + t;
        const uint64_t i = base + q;
        if (i >= n) break;
        if ((bm[q >> 5] >> (q & 31u)) & 1u) {
            const uint32_t r = run_of(bm, wpre, c0, q);
            const Key128 key = k[i];
            gstart[r] = (uint32_t)i;
            glo[r] = key.lo;
            ghi[r] = key.hi;
        }
    }
}

__global__ __launch_bounds__(256) void k_iota_u32(uint32_t* p, uint32_t m)
{
    for (uint32_t j = blockIdx.x * 256 + threadIdx.x; j < m; j += gridDim.x * 256) p[j] = j;
}

// out[j] = src[idx[j]] for j < m (a word of every run, in a run order).
__global__ __launch_bounds__(256) void k_gather_u64_u32(const uint64_t* src, const uint32_t* idx, uint32_t m,
                                                         uint64_t* out)
{
    for (uint32_t j = blockIdx.x * 256 + threadIdx.x; j < m; j += gridDim.x * 256) out[j] = src[idx[j]];
}

// Lengths of the runs in key order: len[j] of run order[j].
__global__ __launch_bounds__(256) void k_runs_lens(const uint32_t* order, const uint32_t* gstart, uint32_t m,
                                                   uint64_t n, uint32_t* len)
{
    for (uint32_t j = blockIdx.x * 256 + threadIdx.x; j < m; j += gridDim.x * 256) {
        const uint32_t g = order[j];
        const uint64_t end = g + 1 < m ? gstart[g + 1] : n;
        len[j] = (uint32_t)(end - gstart[g]);
    }
}

// Per chunk of 4096 entries of len: its sum (for the scan over chunks).
__global__ __launch_bounds__(256) void k_sum_chunks_u32(const uint32_t* len, uint32_t m, uint32_t* csum)
{
    __shared__ uint32_t tmp[20];
    const uint64_t j0 = (uint64_t)blockIdx.x * kRunChunk + (uint64_t)threadIdx.x * kRunPer;
    uint32_t c = 0;
    for (uint32_t q = 0; q < kRunPer; ++q)
        if (j0 + q < m) c += len[j0 + q];
    uint32_t tot = 0;
    (void)block_excl_scan<256>(c, tmp, &tot);
    if (threadIdx.x == 0) csum[blockIdx.x] = tot;
}

// Destination of every run: dest[order[j]] = the lengths of the runs before
// position j of the key order (csum: the chunks' exclusive prefix).
__global__ __launch_bounds__(256) void k_runs_dest(const uint32_t* len, const uint32_t* order, uint32_t m,
                                                   const uint32_t* csum, uint32_t* dest)
{
    __shared__ uint32_t tmp[20];
    const uint64_t j0 = (uint64_t)blockIdx.x * kRunChunk + (uint64_t)threadIdx.x * kRunPer;
    uint32_t c = 0;
    for (uint32_t q = 0; q < kRunPer; ++q)
        if (j0 + q < m) c += len[j0 + q];
    uint32_t p = csum[blockIdx.x] + block_excl_scan<256>(c, tmp, nullptr);
    for (uint32_t q = 0; q < kRunPer; ++q) {
        const uint64_t j = j0 + q;
        if (j >= m) break;
        dest[order[j]] = p;
        p += len[j];
    }
}

// Every record to its run's place, position dest[r] + (i - gstart[r]), one
// chunk per block: the run number r comes from the chunk's stored run-start
// bitmap (no per-record run array).
template <typename V>
__global__ __launch_bounds__(256) void k_runs_scatter(const Key128* gk, const V* gv, uint64_t n, const uint32_t* cbase,
                                                      const uint32_t* bits, const uint32_t* gstart,
                                                      const uint32_t* dest, Key128* ok, V* ov)
{
    __shared__ uint32_t bm[kRunWords], wpre[kRunWords], tmp[20];
    Key128 kk[kRunPer];
    V vv[kRunPer];
    const uint64_t base = (uint64_t)blockIdx.x * kRunChunk;
    const uint32_t t = threadIdx.x;
#pragma unroll
    for (uint32_t j = 0; j < kRunPer; ++j) {
        const uint64_t i = base + j * 256 + t;
        kk[j] = i < n ? gk[i] : Key128{0ull, 0ull};
        vv[j] = i < n ? gv[i] : (V)0;
    }
    load_run_bitmap(bits, bm, wpre, tmp);
    const uint32_t c0 = cbase[blockIdx.x];
#pragma unroll
    for (uint32_t j = 0; j < kRunPer; ++j) {
        const uint32_t q = j * 256 + t;
        const uint64_t i = base + q;
        if (i >= n) break;
        const uint32_t r = run_of(bm, wpre, c0, q);
        const uint64_t p = (uint64_t)dest[r] + (i - gstart[r]);
        ok[p] = kk[j];
        ov[p] = vv[j];
    }
}

}  // namespace ssd
