// Device side of the semisort engine: data structures, wave primitives and the
// kernels of one recursion level (Algorithm 1 of Dong et al., SPAA 2023),
// written for gfx950 (CDNA4, wave64, 160 KB LDS per CU).
//
// Layout conventions
//   * keys[] (u64) and vals[] (u32 or u64) are separate arrays (SoA).
//   * A recursion level holds a list of subproblems (Seg).  Every kernel of
//     the level runs over all of them at once: a block finds its subproblem
//     by binary search over the subproblems' first tile / chunk.
//   * The counting matrix of Section 3.2 is stored one row per subarray
//     ("tile"), row stride kNbStride u32, and is overwritten in place by the
//     column-major prefix X (absolute output positions).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssd {

constexpr uint32_t kHeavyMax = 512;          // n_H cap per subproblem
constexpr uint32_t kLightBitsMax = 10;       // n_L <= 2^10
constexpr uint32_t kNbStride = (1u << kLightBitsMax) + kHeavyMax;  // 1536 buckets max
constexpr uint32_t kSampleMax = 16384;       // |S| cap (LDS bitonic capacity)
constexpr uint32_t kHeavySlotsMax = 1024;    // heavy table slots (load <= 1/2)
constexpr uint32_t kAlphaMax = 4096;         // largest base case held in LDS
constexpr uint32_t kChunk = 32;              // subarrays per scan chunk
constexpr uint32_t kCopyChunk = 65536;       // records per copy job
constexpr uint32_t kBucketGroups = kNbStride / 64;  // 24 column groups in the bucket scan
constexpr uint16_t kEmpty16 = 0xFFFF;
constexpr uint32_t kEmpty32 = 0xFFFFFFFFu;
constexpr uint32_t kJobCopy = 0x80000000u;

// device status bits
constexpr uint32_t kStatusSizeMismatch = 1u;   // bucket sizes do not add up to the subproblem
constexpr uint32_t kStatusScatterRange = 2u;   // a distribution target fell outside its subproblem
constexpr uint32_t kStatusBaseIndex = 4u;      // a base-case permutation entry out of range

struct Seg {
    uint32_t start;    // absolute first record
    uint32_t len;
    uint32_t ibase;    // first record of the instance the subproblem belongs to
    uint32_t tile0;    // first tile of the subproblem in the level's tile list
    uint32_t chunk0;   // first scan chunk
    uint32_t ntiles;
    uint16_t nl_bits;  // light id bits b (n_L = 2^b)
    uint16_t shift;    // first hash bit of the light id
    uint16_t nheavy;   // n_H, written by the sampling kernel
    uint16_t hlog2;    // log2 heavy-table slots, 0 when n_H = 0
};
static_assert(sizeof(Seg) == 32, "Seg layout");

struct Job {
    uint32_t start;
    uint32_t len;      // kJobCopy bit set: plain copy to the output
};

struct LevelInfo {
    uint32_t nsegs;         // subproblems emitted for the next level
    uint32_t njobs;         // jobs emitted by this level
    uint32_t tiles;         // tiles of the next level
    uint32_t chunks;        // scan chunks of the next level
    uint32_t tile;          // subarray size of the next level
    uint32_t status;        // device-detected errors
    uint32_t pad0, pad1;
};

struct LevelArgs {
    const uint64_t* src_keys;
    const void* src_vals;
    uint64_t* dst_keys;
    void* dst_vals;
    Seg* segs;
    uint32_t nsegs;
    uint32_t tile;
    uint32_t* C;           // [tiles][kNbStride]
    uint32_t* P;           // [chunks][kNbStride]
    uint32_t* tot;         // [nsegs][kNbStride]
    uint32_t* bstart;      // [nsegs][kNbStride + 1]
    uint64_t* heavy_list;  // [nsegs][kHeavyMax]  heavy hashes in id order
    uint64_t* tab_h;       // [nsegs][kHeavySlotsMax]
    uint16_t* tab_id;      // [nsegs][kHeavySlotsMax]
    LevelInfo* info;
    uint64_t seed;
    uint32_t level;
    uint32_t sample_mult;
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

// SplitMix64's output function (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// Table slot from a hash: Fibonacci hashing keeps the top bits of h * 2^64/phi,
// so identity-hashed small integers still spread.
__device__ __forceinline__ uint32_t fib_slot(uint64_t h, uint32_t log2slots)
{
    return (uint32_t)((h * 0x9e3779b97f4a7c15ULL) >> (64 - log2slots));
}

// GetBucketId (Algorithm 1): heavy id from the heavy table, else the light id
// from nl_bits bits of the hash starting at `shift`.
__device__ __forceinline__ uint32_t bucket_of(uint64_t h, const uint64_t* th, const uint16_t* tid,
                                              uint32_t hlog2, uint32_t shift, uint32_t lmask)
{
    if (hlog2) {
        const uint32_t mask = (1u << hlog2) - 1;
        uint32_t s = fib_slot(h, hlog2);
        while (true) {
            uint16_t id = tid[s];
            if (id == kEmpty16) break;
            if (th[s] == h) return id;
            s = (s + 1) & mask;
        }
    }
    return (uint32_t)(h >> shift) & lmask;
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
// about alpha/2 records (at least 1 bit, at most kLightBitsMax and the hash
// bits left).
__host__ __device__ __forceinline__ uint32_t choose_nl(uint32_t len, uint32_t alpha, uint32_t cap,
                                                       uint32_t shift)
{
    uint32_t target = alpha / 2 ? alpha / 2 : 1;
    uint32_t q = (len + target - 1) / target;
    uint32_t nl = ceil_log2_u32(q);
    if (nl < 1) nl = 1;
    if (nl > cap) nl = cap;
    if (nl > 64 - shift) nl = 64 - shift;
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
// sorted by hash in LDS; keys seen at least ceil(ln n') times are heavy and get
// ids n_L, n_L + 1, ... in ascending hash order; an open-addressing heavy
// table is built for the later passes.  One block per subproblem.

template <int MODE>
__global__ __launch_bounds__(1024) void k_sample_heavy(LevelArgs a)
{
    constexpr int BS = 1024;
    __shared__ uint64_t smp[kSampleMax];
    __shared__ uint64_t hv[kHeavyMax];
    __shared__ uint32_t owner[kHeavySlotsMax];
    __shared__ uint32_t tmp[20];
    __shared__ uint32_t sh_s, sh_tau;

    const uint32_t sid = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const Seg sg = a.segs[sid];
    if (tid == 0) {
        const double L = log((double)sg.len);
        double sd = ceil((double)a.sample_mult * L);
        uint32_t s = sg.len < 2 ? 0u : (uint32_t)sd;
        if (s > kSampleMax) s = kSampleMax;
        sh_s = s;
        sh_tau = sg.len < 3 ? 1u : (uint32_t)ceil(L);
    }
    __syncthreads();
    const uint32_t s = sh_s, tau = sh_tau;
    uint32_t P = 2;
    while (P < s) P <<= 1;

    const uint64_t golden = 0x9e3779b97f4a7c15ULL;
    const uint64_t k0 = splitmix_mix(a.seed + golden * ((uint64_t)a.level + 1));
    const uint64_t k1 = splitmix_mix(k0 ^ (uint64_t)(sg.start - sg.ibase));
    for (uint32_t i = tid; i < P; i += BS) {
        uint64_t v = ~0ull;
        if (i < s) {
            uint64_t r = splitmix_mix(k1 + golden * ((uint64_t)i + 1));
            uint64_t idx = __umul64hi(r, (uint64_t)sg.len);
            v = user_hash<MODE>(a.src_keys[(uint64_t)sg.start + idx]);
        }
        smp[i] = v;
    }
    __syncthreads();

    // bitonic sort of smp[0, P), ascending
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t t = tid; t < (P >> 1); t += BS) {
                const uint32_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                const uint32_t l = i + j;
                const bool up = (i & k) == 0;
                const uint64_t x = smp[i], y = smp[l];
                if ((x > y) == up) {
                    smp[i] = y;
                    smp[l] = x;
                }
            }
            __syncthreads();
        }
    }

    // heavy run starts: a run of equal hashes of length >= tau among the s real samples
    const uint32_t per = (s + BS - 1) / BS;
    const uint32_t lo = tid * per;
    const uint32_t hi = lo + per < s ? lo + per : s;
    uint32_t cnt = 0;
    for (uint32_t i = lo; i < hi; ++i) {
        const bool start = (i == 0) || smp[i] != smp[i - 1];
        if (start && i + tau - 1 < s && smp[i + tau - 1] == smp[i]) ++cnt;
    }
    uint32_t total = 0;
    uint32_t id = block_excl_scan<BS>(cnt, tmp, &total);
    const uint32_t nh = total < kHeavyMax ? total : kHeavyMax;
    for (uint32_t i = lo; i < hi; ++i) {
        const bool start = (i == 0) || smp[i] != smp[i - 1];
        if (start && i + tau - 1 < s && smp[i + tau - 1] == smp[i]) {
            if (id < kHeavyMax) {
                hv[id] = smp[i];
                a.heavy_list[(size_t)sid * kHeavyMax + id] = smp[i];
            }
            ++id;
        }
    }
    uint32_t hlog2 = 0;
    if (nh) {
        hlog2 = ceil_log2_u32(2 * nh);
        if (hlog2 < 4) hlog2 = 4;
    }
    const uint32_t slots = nh ? (1u << hlog2) : 0u;
    for (uint32_t i = tid; i < slots; i += BS) owner[i] = kEmpty32;
    __syncthreads();
    for (uint32_t t = tid; t < nh; t += BS) {
        const uint64_t h = hv[t];
        uint32_t sl = fib_slot(h, hlog2);
        while (true) {
            uint32_t old = atomicCAS(&owner[sl], kEmpty32, t);
            if (old == kEmpty32) break;
            sl = (sl + 1) & (slots - 1);
        }
    }
    __syncthreads();
    const uint32_t nL = 1u << sg.nl_bits;
    for (uint32_t i = tid; i < slots; i += BS) {
        const uint32_t o = owner[i];
        a.tab_h[(size_t)sid * kHeavySlotsMax + i] = o != kEmpty32 ? hv[o] : 0ull;
        a.tab_id[(size_t)sid * kHeavySlotsMax + i] = o != kEmpty32 ? (uint16_t)(nL + o) : kEmpty16;
    }
    if (tid == 0) {
        a.segs[sid].nheavy = (uint16_t)nh;
        a.segs[sid].hlog2 = (uint16_t)hlog2;
    }
}

// ================================================================ Step 2a
// Counting pass (Section 3.2): per subarray, sequential over its records in
// the paper; here one block per subarray with LDS counters.  Counting is
// order-free, so plain LDS atomics suffice.

template <int MODE>
__global__ __launch_bounds__(1024) void k_count(LevelArgs a)
{
    constexpr int BS = 1024;
    __shared__ uint32_t cnt[kNbStride];
    __shared__ uint64_t th[kHeavySlotsMax];
    __shared__ uint16_t tidh[kHeavySlotsMax];

    const uint32_t t = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t sid = find_by_tile(a.segs, a.nsegs, t);
    const Seg sg = a.segs[sid];
    const uint32_t lt = t - sg.tile0;
    const uint64_t r0 = (uint64_t)sg.start + (uint64_t)lt * a.tile;
    const uint64_t send = (uint64_t)sg.start + sg.len;
    const uint64_t r1 = r0 + a.tile < send ? r0 + a.tile : send;
    const uint32_t nL = 1u << sg.nl_bits;
    const uint32_t nb = nL + sg.nheavy;
    const uint32_t hlog2 = sg.hlog2;
    const uint32_t slots = hlog2 ? (1u << hlog2) : 0u;

    for (uint32_t b = tid; b < nb; b += BS) cnt[b] = 0;
    for (uint32_t i = tid; i < slots; i += BS) {
        th[i] = a.tab_h[(size_t)sid * kHeavySlotsMax + i];
        tidh[i] = a.tab_id[(size_t)sid * kHeavySlotsMax + i];
    }
    __syncthreads();

    const uint32_t shift = sg.shift;
    const uint32_t lmask = nL - 1;
    const uint64_t* keys = a.src_keys;
    uint64_t i = r0 + tid;
    for (; i + 3 * BS < r1; i += 4 * BS) {
        uint64_t k0 = keys[i], k1 = keys[i + BS], k2 = keys[i + 2 * BS], k3 = keys[i + 3 * BS];
        atomicAdd(&cnt[bucket_of(user_hash<MODE>(k0), th, tidh, hlog2, shift, lmask)], 1u);
        atomicAdd(&cnt[bucket_of(user_hash<MODE>(k1), th, tidh, hlog2, shift, lmask)], 1u);
        atomicAdd(&cnt[bucket_of(user_hash<MODE>(k2), th, tidh, hlog2, shift, lmask)], 1u);
        atomicAdd(&cnt[bucket_of(user_hash<MODE>(k3), th, tidh, hlog2, shift, lmask)], 1u);
    }
    for (; i < r1; i += BS)
        atomicAdd(&cnt[bucket_of(user_hash<MODE>(keys[i]), th, tidh, hlog2, shift, lmask)], 1u);
    __syncthreads();
    uint32_t* row = a.C + (size_t)t * kNbStride;
    for (uint32_t b = tid; b < nb; b += BS) row[b] = cnt[b];
}

// ================================================================ Step 2b
// Column-major prefix X of the counting matrix (Algorithm 1): per bucket, the
// records of all earlier buckets plus that bucket's records in earlier
// subarrays.  Four passes over the rows: chunk sums, a scan over chunks per
// bucket, bucket starts per subproblem, and the fill of X.

__global__ __launch_bounds__(256) void k_scan_chunks(LevelArgs a)
{
    const uint32_t ch = blockIdx.x;
    const uint32_t sid = find_by_chunk(a.segs, a.nsegs, ch);
    const Seg sg = a.segs[sid];
    const uint32_t lc = ch - sg.chunk0;
    const uint32_t t0 = sg.tile0 + lc * kChunk;
    const uint32_t tend = sg.tile0 + sg.ntiles;
    const uint32_t t1 = t0 + kChunk < tend ? t0 + kChunk : tend;
    const uint32_t nb = (1u << sg.nl_bits) + sg.nheavy;
    for (uint32_t b = threadIdx.x; b < nb; b += 256) {
        uint32_t s = 0;
        for (uint32_t t = t0; t < t1; ++t) s += a.C[(size_t)t * kNbStride + b];
        a.P[(size_t)ch * kNbStride + b] = s;
    }
}

__global__ __launch_bounds__(1024) void k_scan_buckets(LevelArgs a)
{
    __shared__ uint32_t part[16][64];
    const uint32_t sid = blockIdx.x / kBucketGroups;
    const uint32_t bg = blockIdx.x % kBucketGroups;
    const Seg sg = a.segs[sid];
    const uint32_t nb = (1u << sg.nl_bits) + sg.nheavy;
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

__global__ __launch_bounds__(1024) void k_scan_offsets(LevelArgs a)
{
    __shared__ uint32_t tmp[20];
    const uint32_t sid = blockIdx.x;
    const Seg sg = a.segs[sid];
    const uint32_t nb = (1u << sg.nl_bits) + sg.nheavy;
    const uint32_t b0 = 2 * threadIdx.x, b1 = b0 + 1;
    const uint32_t v0 = b0 < nb ? a.tot[(size_t)sid * kNbStride + b0] : 0u;
    const uint32_t v1 = b1 < nb ? a.tot[(size_t)sid * kNbStride + b1] : 0u;
    uint32_t total = 0;
    const uint32_t base = block_excl_scan<1024>(v0 + v1, tmp, &total);
    uint32_t* bs = a.bstart + (size_t)sid * (kNbStride + 1);
    if (b0 < nb) bs[b0] = sg.start + base;
    if (b1 < nb) bs[b1] = sg.start + base + v0;
    if (threadIdx.x == 0) {
        bs[nb] = sg.start + sg.len;
        if (total != sg.len) atomicOr(&a.info->status, kStatusSizeMismatch);
    }
}

__global__ __launch_bounds__(256) void k_scan_fill(LevelArgs a)
{
    const uint32_t ch = blockIdx.x;
    const uint32_t sid = find_by_chunk(a.segs, a.nsegs, ch);
    const Seg sg = a.segs[sid];
    const uint32_t lc = ch - sg.chunk0;
    const uint32_t t0 = sg.tile0 + lc * kChunk;
    const uint32_t tend = sg.tile0 + sg.ntiles;
    const uint32_t t1 = t0 + kChunk < tend ? t0 + kChunk : tend;
    const uint32_t nb = (1u << sg.nl_bits) + sg.nheavy;
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

// ================================================================ Step 2c
// Distribution (Section 3.2): each subarray, in order, moves every record to
// T[X[i][id]++].  One block per subarray walks it in sub-tiles of W*64*E
// records; each wave ranks its contiguous chunk stably (ballot match plus
// per-wave LDS counters), the block turns ranks into bucket-grouped LDS
// positions, and the staged sub-tile is written out so that consecutive
// threads write consecutive addresses of a bucket's run.  Keys go first,
// then values through the same staging buffer.

template <int MODE, typename V, int W, int E>
__global__ __launch_bounds__(W * 64) void k_distribute(LevelArgs a)
{
    constexpr int BS = W * 64;
    constexpr int SUB = BS * E;
    __shared__ uint64_t th[kHeavySlotsMax];
    __shared__ uint16_t tidh[kHeavySlotsMax];
    __shared__ uint32_t gbase[kNbStride];
    __shared__ uint32_t lst[kNbStride];
    __shared__ uint32_t ltot[kNbStride];
    __shared__ uint16_t wc[W * kNbStride];
    __shared__ uint64_t stage[SUB];
    __shared__ uint16_t stage_b[SUB];
    __shared__ uint32_t tmp[20];

    const uint32_t t = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, w = tid >> 6;
    const uint32_t sid = find_by_tile(a.segs, a.nsegs, t);
    const Seg sg = a.segs[sid];
    const uint32_t lt = t - sg.tile0;
    const uint64_t r0 = (uint64_t)sg.start + (uint64_t)lt * a.tile;
    const uint64_t send = (uint64_t)sg.start + sg.len;
    const uint64_t r1 = r0 + a.tile < send ? r0 + a.tile : send;
    const uint32_t nL = 1u << sg.nl_bits;
    const uint32_t nb = nL + sg.nheavy;
    const uint32_t nbits = 32 - __clz(nb - 1);
    const uint32_t hlog2 = sg.hlog2;
    const uint32_t slots = hlog2 ? (1u << hlog2) : 0u;
    const uint32_t shift = sg.shift;
    const uint32_t lmask = nL - 1;
    const V* src_vals = (const V*)a.src_vals;
    V* dst_vals = (V*)a.dst_vals;
    V* stage_v = (V*)stage;

    for (uint32_t i = tid; i < slots; i += BS) {
        th[i] = a.tab_h[(size_t)sid * kHeavySlotsMax + i];
        tidh[i] = a.tab_id[(size_t)sid * kHeavySlotsMax + i];
    }
    for (uint32_t b = tid; b < nb; b += BS) gbase[b] = a.C[(size_t)t * kNbStride + b];

    for (uint64_t sub = r0; sub < r1; sub += SUB) {
        for (uint32_t i = tid; i < W * nb; i += BS) wc[i] = 0;
        __syncthreads();

        uint64_t k[E];
        V v[E];
        uint32_t bk[E], pos[E];
        const uint64_t base_i = sub + (uint64_t)w * 64 * E + lane;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint64_t i = base_i + (uint64_t)e * 64;
            const bool valid = i < r1;
            k[e] = valid ? a.src_keys[i] : 0ull;
            v[e] = valid ? src_vals[i] : (V)0;
        }
#pragma unroll
        for (int e = 0; e < E; ++e)
            bk[e] = bucket_of(user_hash<MODE>(k[e]), th, tidh, hlog2, shift, lmask);
        uint16_t* wcw = wc + w * nb;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const bool valid = base_i + (uint64_t)e * 64 < r1;
            pos[e] = wave_rank(bk[e], valid, nbits, wcw);
        }
        __syncthreads();

        // per-bucket prefix over waves and the sub-tile's bucket totals
        for (uint32_t b = tid; b < nb; b += BS) {
            uint32_t run = 0;
            for (int ww = 0; ww < W; ++ww) {
                const uint32_t c = wc[ww * nb + b];
                wc[ww * nb + b] = (uint16_t)run;
                run += c;
            }
            ltot[b] = run;
        }
        __syncthreads();
        {
            // exclusive scan of ltot over the nb buckets, contiguous pieces per thread
            const uint32_t per = (nb + BS - 1) / BS;
            const uint32_t b0 = tid * per;
            uint32_t s = 0;
            for (uint32_t j = 0; j < per; ++j)
                if (b0 + j < nb) s += ltot[b0 + j];
            uint32_t run = block_excl_scan<BS>(s, tmp, nullptr);
            for (uint32_t j = 0; j < per; ++j)
                if (b0 + j < nb) {
                    lst[b0 + j] = run;
                    run += ltot[b0 + j];
                }
        }
        __syncthreads();

#pragma unroll
        for (int e = 0; e < E; ++e) {
            const bool valid = base_i + (uint64_t)e * 64 < r1;
            if (valid) {
                const uint32_t p = lst[bk[e]] + wc[w * nb + bk[e]] + pos[e];
                pos[e] = p;
                stage[p] = k[e];
                stage_b[p] = (uint16_t)bk[e];
            }
        }
        __syncthreads();
        const uint32_t m = (uint32_t)((r1 - sub) < (uint64_t)SUB ? (r1 - sub) : (uint64_t)SUB);
        bool out_of_range = false;
        for (uint32_t j = tid; j < m; j += BS) {
            const uint32_t b = stage_b[j];
            const uint32_t d = gbase[b] + (j - lst[b]);
            if (d - sg.start < sg.len) a.dst_keys[d] = stage[j];
            else out_of_range = true;
        }
        if (out_of_range) atomicOr(&a.info->status, kStatusScatterRange);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const bool valid = base_i + (uint64_t)e * 64 < r1;
            if (valid) stage_v[pos[e]] = v[e];
        }
        __syncthreads();
        for (uint32_t j = tid; j < m; j += BS) {
            const uint32_t b = stage_b[j];
            const uint32_t d = gbase[b] + (j - lst[b]);
            if (d - sg.start < sg.len) dst_vals[d] = stage_v[j];
        }
        __syncthreads();
        for (uint32_t b = tid; b < nb; b += BS) gbase[b] += ltot[b];
    }
}

// ================================================================ Step 3 planning
// After a level's distribution, every bucket of every subproblem becomes one
// of: a subproblem of the next level (light, >= alpha records: the recursive
// call of Algorithm 1), a base-case job (light, 2 .. alpha-1 records), a copy
// job (a bucket that is already final but sits in T, Section 3.4), or nothing.
// Heavy buckets are final (Section 3.3).  Appends are aggregated per block.

struct PlanArgs {
    const Seg* segs;
    uint32_t nsegs;
    const uint32_t* bstart;
    Seg* next;
    uint32_t next_cap;
    Job* jobs;
    uint32_t job_cap;
    LevelInfo* info;
    uint32_t alpha;
    uint32_t dst_is_out;
};

__device__ __forceinline__ void plan_bucket(const PlanArgs& p, const Seg& sg, uint32_t b, uint32_t nL,
                                            uint32_t& nseg, uint32_t& njob, bool emit,
                                            uint32_t& seg_at, uint32_t& job_at)
{
    const uint32_t* bs = p.bstart + (size_t)(&sg - p.segs) * (kNbStride + 1);
    const uint32_t st = bs[b];
    const uint32_t sz = bs[b + 1] - st;
    if (sz == 0) return;
    const uint32_t shift2 = sg.shift + sg.nl_bits;
    const bool heavy = b >= nL;
    const bool all_bits_used = shift2 >= 64;
    bool final_copy = false;
    if (heavy || sz == 1 || (all_bits_used && sz >= p.alpha)) {
        final_copy = !p.dst_is_out;
    } else if (sz >= p.alpha) {
        if (emit && seg_at < p.next_cap) {
            Seg ns;
            ns.start = st;
            ns.len = sz;
            ns.ibase = sg.ibase;
            ns.tile0 = ns.chunk0 = ns.ntiles = 0;
            ns.nl_bits = (uint16_t)choose_nl(sz, p.alpha, kLightBitsMax, shift2);
            ns.shift = (uint16_t)shift2;
            ns.nheavy = 0;
            ns.hlog2 = 0;
            p.next[seg_at] = ns;
        }
        ++seg_at;
        ++nseg;
        return;
    } else {
        if (emit && job_at < p.job_cap) p.jobs[job_at] = Job{st, sz};
        ++job_at;
        ++njob;
        return;
    }
    if (final_copy) {
        for (uint32_t o = 0; o < sz; o += kCopyChunk) {
            const uint32_t l = sz - o < kCopyChunk ? sz - o : kCopyChunk;
            if (emit && job_at < p.job_cap) p.jobs[job_at] = Job{st + o, l | kJobCopy};
            ++job_at;
            ++njob;
        }
    }
}

__global__ __launch_bounds__(256) void k_plan(PlanArgs p)
{
    __shared__ uint32_t tmp[20];
    __shared__ uint32_t sh_seg, sh_job;
    const Seg& sg = p.segs[blockIdx.x];
    const uint32_t nL = 1u << sg.nl_bits;
    const uint32_t nb = nL + sg.nheavy;
    uint32_t nseg = 0, njob = 0, dummy_s = 0, dummy_j = 0;
    for (uint32_t b = threadIdx.x; b < nb; b += 256)
        plan_bucket(p, sg, b, nL, nseg, njob, false, dummy_s, dummy_j);
    uint32_t tot_s = 0, tot_j = 0;
    uint32_t off_s = block_excl_scan<256>(nseg, tmp, &tot_s);
    uint32_t off_j = block_excl_scan<256>(njob, tmp, &tot_j);
    if (threadIdx.x == 0) {
        sh_seg = tot_s ? atomicAdd(&p.info->nsegs, tot_s) : 0u;
        sh_job = tot_j ? atomicAdd(&p.info->njobs, tot_j) : 0u;
    }
    __syncthreads();
    uint32_t seg_at = sh_seg + off_s, job_at = sh_job + off_j;
    nseg = njob = 0;
    for (uint32_t b = threadIdx.x; b < nb; b += 256)
        plan_bucket(p, sg, b, nL, nseg, njob, true, seg_at, job_at);
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
    }
}

// ================================================================ Step 3
// Local refining base case for semisort_= (Section 3.3).  The paper packs a
// sequential chained hash table in table order.  Here one block per bucket:
// the keys go to LDS, an LDS hash table (open addressing, CAS on slot
// owners, keys compared through the owner's index) yields f(i) = the first
// index of record i's key, and a stable two-pass LDS radix sort on f(i)
// groups equal keys in order of first occurrence while keeping input order
// inside a group.  Copy jobs move final buckets from T to the output.

template <int MODE, typename V>
__global__ __launch_bounds__(512) void k_finish(const Job* jobs, const uint64_t* src_keys,
                                                const V* src_vals, uint64_t* out_keys, V* out_vals,
                                                LevelInfo* info)
{
    constexpr int W = 8, BS = 512, E = kAlphaMax / BS;  // 8 records per thread
    __shared__ uint64_t kl[kAlphaMax];
    __shared__ uint32_t tab[2 * kAlphaMax];   // slot owners, then the two sort buffers
    __shared__ uint32_t fmin[2 * kAlphaMax];
    __shared__ uint16_t wc[W * 128];
    __shared__ uint32_t dtot[128];
    __shared__ uint32_t dst_[128];
    __shared__ uint32_t tmp[20];

    const Job j = jobs[blockIdx.x];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    const uint32_t len = j.len & ~kJobCopy;
    const uint64_t start = j.start;
    if (j.len & kJobCopy) {
        for (uint32_t i = tid; i < len; i += BS) {
            out_keys[start + i] = src_keys[start + i];
            out_vals[start + i] = src_vals[start + i];
        }
        return;
    }
    const uint32_t m = len;  // 2 .. kAlphaMax-1
    const uint32_t lg = ceil_log2_u32(2 * m) < 6 ? 6 : ceil_log2_u32(2 * m);
    const uint32_t slots = 1u << lg, smask = slots - 1;
    for (uint32_t i = tid; i < m; i += BS) kl[i] = src_keys[start + i];
    for (uint32_t i = tid; i < slots; i += BS) {
        tab[i] = kEmpty32;
        fmin[i] = kEmpty32;
    }
    __syncthreads();

    uint32_t myslot[E], f[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t i = w * 64 * E + e * 64 + lane;
        myslot[e] = 0;
        if (i < m) {
            const uint64_t key = kl[i];
            uint32_t sl = fib_slot(user_hash<MODE>(key), lg);
            while (true) {
                uint32_t o = tab[sl];
                if (o == kEmpty32) {
                    o = atomicCAS(&tab[sl], kEmpty32, i);
                    if (o == kEmpty32) break;
                }
                if (kl[o] == key) break;
                sl = (sl + 1) & smask;
            }
            myslot[e] = sl;
            atomicMin(&fmin[sl], i);
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) f[e] = fmin[myslot[e]];
    __syncthreads();

    uint32_t* A = tab;              // after pass 1
    uint32_t* B = tab + kAlphaMax;  // after pass 2
    // element carried through the sort: (index << 16) | f
    uint32_t el[E];
#pragma unroll
    for (int e = 0; e < E; ++e) el[e] = ((w * 64 * E + e * 64 + lane) << 16) | (f[e] & 0xFFFFu);

#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        const uint32_t sh = pass ? 7u : 0u;
        const uint32_t nbits = pass ? 5u : 7u;
        for (uint32_t i = tid; i < W * 128; i += BS) wc[i] = 0;
        __syncthreads();
        uint32_t rk[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t q = w * 64 * E + e * 64 + lane;
            const uint32_t d = ((el[e] & 0xFFFFu) >> sh) & ((1u << nbits) - 1);
            rk[e] = wave_rank(d, q < m, nbits, wc + w * 128);
        }
        __syncthreads();
        if (tid < 128) {
            uint32_t run = 0;
            for (int ww = 0; ww < W; ++ww) {
                const uint32_t c = wc[ww * 128 + tid];
                wc[ww * 128 + tid] = (uint16_t)run;
                run += c;
            }
            dtot[tid] = run;
        }
        __syncthreads();
        const uint32_t dv = tid < 128 ? dtot[tid] : 0u;
        const uint32_t ds = block_excl_scan<BS>(dv, tmp, nullptr);
        if (tid < 128) dst_[tid] = ds;
        __syncthreads();
        uint32_t* out = pass ? B : A;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t q = w * 64 * E + e * 64 + lane;
            if (q < m) {
                const uint32_t d = ((el[e] & 0xFFFFu) >> sh) & ((1u << nbits) - 1);
                out[dst_[d] + wc[w * 128 + d] + rk[e]] = el[e];
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

    // gather, then write (the output may be the source: in-place within the block)
    uint64_t ok[E];
    V ov[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t q = tid + e * BS;
        if (q < m) {
            uint32_t i = B[q] >> 16;
            if (i >= m) {
                atomicOr(&info->status, kStatusBaseIndex);
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
            out_keys[start + q] = ok[e];
            out_vals[start + q] = ov[e];
        }
    }
}

// Offsets and heavy list of a single-subproblem level, for inspection.
__global__ void k_export_partition(const uint32_t* bstart, const Seg* segs, const uint64_t* heavy_list,
                                   uint64_t* offsets_out, uint64_t* heavy_out)
{
    const Seg sg = segs[0];
    const uint32_t nb = (1u << sg.nl_bits) + sg.nheavy;
    for (uint32_t b = threadIdx.x; b <= nb; b += blockDim.x) offsets_out[b] = bstart[b] - sg.start;
    for (uint32_t h = threadIdx.x; h < sg.nheavy; h += blockDim.x) heavy_out[h] = heavy_list[h];
}

}  // namespace ssd
