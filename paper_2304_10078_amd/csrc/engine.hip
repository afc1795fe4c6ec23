// Host driver and C-ABI of libsemisort_hip.so (declared in include/semisort.h).
//
// The host engine runs Algorithm 1 level by level over a list of subproblems: all
// subproblems of one recursion level are processed by the same kernel
// launches (sampling, counting, scan, distribution), then a planning kernel
// turns every bucket into a next-level subproblem, a base-case job or a copy
// job.  One host synchronization per level reads the sizes of the next level
// (run_semisort_ds instead keeps them on the device for graph capture).
// Buffers alternate between the output and the temporary array T as in the
// in-place optimization of Section 3.4.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cstddef>
#include <functional>
#include <map>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "semisort.h"
#include "ss_device.h"
#include "user_fold.inc"

using namespace ssd;

namespace {

// Stores of lanes without a record go to a sink of 64 lanes of the widest key.
constexpr size_t kSinkBytes = 64 * 16;

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

}  // namespace

// Workspace of ss_semisort_equal_batch_noalloc, for callers that cannot
// allocate: a static device array, one copy per device, held by every device
// the library runs on until the process ends.  Host code never passes its
// name to a kernel (on the host the name is only a stand-in); it uses the
// device address looked up once per device.
constexpr size_t kScratchBytes = 64ull << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on `device`, which must be current.
hipError_t scratch_address(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

struct ss_ctx {
    int device = 0;
    int ncu = 1;  // compute units of the device (persistent grids)
    hipStream_t stream = nullptr;
    std::string err;
    DevBuf t_keys, t_vals;
    DevBuf segs[2];
    DevBuf jobs;
    DevBuf C, P, tot, bstart, heavy_list, tab_h, tab_id, bids, sink, bfin;
    DevBuf hsum, rflag, bcnt, mdev;  // collect-reduce and histogram
    DevBuf bkey;                     // keys of one-key buckets
    DevBuf hrep;                     // 128-bit keys: one sampled key per heavy id
    DevBuf wl_gk, wl_gv, wl_chunk, wl_desc;  // semisort_< of 128-bit keys: grouped records, runs
    DevBuf top;                      // two most sampled heavy buckets per subproblem
    DevBuf fills[2];                 // key-fill job lists (alternating levels)
    uint32_t fill_cap[2] = {0, 0};
    hipStream_t aux = nullptr;       // second stream: key fills overlap the next level
    hipEvent_t fill_done[2] = {nullptr, nullptr};
    hipEvent_t fill_fork[2] = {nullptr, nullptr};  // device-sized levels: fills start after the planning
    hipEvent_t plan_ev = nullptr;    // the level's plan has been read back (planning ahead of the distribution)
    DevBuf info;
    LevelInfo* info_host = nullptr;  // pinned
    DevBuf ds_jobs, ds_info, ds_q;   // device-sized batches: job lists, per-level counts, queue counters
    DevBuf tr_keys, tr_vals, tr_sorted, tr_min;  // graph transpose: records, sorted endpoints, chunk minima
    DevBuf pos;                      // record positions (first / last collect-reduce)
    DevBuf pk_k, pk_v, po_k, po_v;   // ss_batch: packed inputs and outputs
    DevBuf pack_tab, pack_rank;      // ss_batch: packed job table, first result rank of every job
    PackJob* pack_stage = nullptr;   // pinned staging of the packed job table
    size_t pack_stage_cap = 0;
    hipEvent_t stage_ev = nullptr;   // last copy out of a pinned staging buffer
    size_t ws_cap = 0;               // workspace cap (0: none), from ss_create
    size_t ws_held = 0;              // bytes of workspace held now
    void* scratch = nullptr;         // device address of the static scratch array on this device
    std::string scratch_err;         // why it has none
    std::vector<Seg> host_segs;
    std::vector<Job> host_jobs[kJobClasses];
    uint32_t job_cap = 0;  // entries per class list
    Seg* seg_stage = nullptr;        // pinned staging for the first level
    size_t seg_stage_cap = 0;
    Job* job_stage = nullptr;
    size_t job_stage_cap = 0;
    int dist_variant = 0;  // distribution kernel shape (ss_set_option)
    uint32_t deep_div = 1;    // sample multiplier divisor below level 0 (ss_set_option)
    uint32_t nl_target = 0;   // adaptive light-bucket target, percent of alpha; 0: per bucketing (ss_set_option)
    uint32_t tile0 = 0, tile_deep = 0;  // tile limits of the first / deeper levels, 0 = tile_max (ss_set_option)
    uint32_t call_tmaxd = 0;            // deeper-level tile limit chosen by the current call (0: Params)
    uint32_t fold_round = 1024;
    std::map<uint64_t, ss_params> tuned;  // autotuned batch parameters by batch class         // block totals per round of the in-order fold's top carry (ss_set_option)
    // kernel timing with HIP events on the context's stream (ss_profile_*)
    bool prof_on = false;
    struct Pending {
        hipEvent_t a, b;
        int kind;
        uint64_t units;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    double prof_ms[SS_PROF_KINDS] = {};
    uint64_t prof_launches[SS_PROF_KINDS] = {};
    uint64_t prof_units[SS_PROF_KINDS] = {};
};

// A caller's monoid compiled for one device: the module of the in-order fold
// kernels instantiated for it.
struct ss_user_monoid {
    int device = -1;
    hipModule_t mod = nullptr;
    hipFunction_t aggr = nullptr, carry_blocks = nullptr, carry_top = nullptr, apply = nullptr;
};

namespace {

ss_status fail(ss_ctx* c, ss_status s, const std::string& msg)
{
    if (c) c->err = msg;
    return s;
}

#define HIP_OR_FAIL(ctx, call)                                                          \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail((ctx), SS_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

// Grows a workspace buffer to at least `bytes` (by half again its size when
// that fits, so buffers that grow level by level are not reallocated each
// time).  With a workspace cap, the context's total must stay within it:
// growth falls back to the exact size, and past the cap the call fails with
// SS_ENOMEM before anything is freed or allocated.
ss_status ensure(ss_ctx* c, DevBuf& b, size_t bytes)
{
    if (bytes <= b.cap) return SS_OK;
    const size_t need = (bytes + 255) & ~(size_t)255;
    size_t want = std::max(bytes, b.cap + b.cap / 2);
    want = (want + 255) & ~(size_t)255;
    const size_t others = c->ws_held - b.cap;
    if (c->ws_cap) {
        if (others + need > c->ws_cap)
            return fail(c, SS_ENOMEM, "the workspace cap of " + std::to_string(c->ws_cap) + " bytes is too small: " +
                                          std::to_string(others + need) + " bytes are needed");
        if (others + want > c->ws_cap) want = need;
    }
    if (b.p) {
        HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
        HIP_OR_FAIL(c, hipFree(b.p));
        b.p = nullptr;
        c->ws_held -= b.cap;
        b.cap = 0;
    }
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(c, SS_ENOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    b.cap = want;
    c->ws_held += want;
    return SS_OK;
}

// Frees a workspace buffer (after the stream's work on it).
ss_status release(ss_ctx* c, DevBuf& b)
{
    if (!b.p) return SS_OK;
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    HIP_OR_FAIL(c, hipFree(b.p));
    c->ws_held -= b.cap;
    b.p = nullptr;
    b.cap = 0;
    return SS_OK;
}

ss_status ensure_pinned(ss_ctx* c, void** p, size_t* cap, size_t bytes)
{
    if (bytes <= *cap) return SS_OK;
    if (*p) {
        HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
        HIP_OR_FAIL(c, hipHostFree(*p));
        *p = nullptr;
        *cap = 0;
    }
    size_t want = std::max<size_t>(bytes, 4096);
    HIP_OR_FAIL(c, hipHostMalloc(p, want, hipHostMallocDefault));
    *cap = want;
    return SS_OK;
}

// The pinned staging buffers are rewritten by the next call: wait for the
// last copy out of them first (stage_mark records it).
ss_status stage_wait(ss_ctx* c)
{
    if (c->stage_ev) HIP_OR_FAIL(c, hipEventSynchronize(c->stage_ev));
    return SS_OK;
}

ss_status stage_mark(ss_ctx* c)
{
    if (c->stage_ev) HIP_OR_FAIL(c, hipEventRecord(c->stage_ev, c->stream));
    return SS_OK;
}

hipEvent_t take_event(ss_ctx* c)
{
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one kernel launch with events when profiling is on.
struct ProfScope {
    ss_ctx* c;
    ss_ctx::Pending p;
    bool on;
    hipStream_t st;
    ProfScope(ss_ctx* ctx, int kind, uint64_t units, hipStream_t stream = nullptr)
        : c(ctx), on(ctx->prof_on), st(stream ? stream : ctx->stream)
    {
        if (!on) return;
        p.kind = kind;
        p.units = units;
        p.a = take_event(c);
        p.b = take_event(c);
        if (!p.a || !p.b) {
            on = false;
            return;
        }
        (void)hipEventRecord(p.a, st);
    }
    ~ProfScope()
    {
        if (!on) return;
        (void)hipEventRecord(p.b, st);
        c->pending.push_back(p);
    }
};

ss_status resolve_profile(ss_ctx* c)
{
    if (c->pending.empty()) return SS_OK;
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    for (auto& p : c->pending) {
        float ms = 0.f;
        HIP_OR_FAIL(c, hipEventElapsedTime(&ms, p.a, p.b));
        c->prof_ms[p.kind] += ms;
        c->prof_launches[p.kind] += 1;
        c->prof_units[p.kind] += p.units;
        c->event_pool.push_back(p.a);
        c->event_pool.push_back(p.b);
    }
    c->pending.clear();
    return SS_OK;
}

// Clears the per-level counters of the device LevelInfo, keeping the sticky status word.
ss_status reset_counters(ss_ctx* c)
{
    HIP_OR_FAIL(c, hipMemsetAsync(c->info.p, 0, (2 + kJobClasses) * sizeof(uint32_t), c->stream));
    HIP_OR_FAIL(c, hipMemsetAsync((char*)c->info.p + offsetof(LevelInfo, records), 0,
                                  3 * sizeof(unsigned long long), c->stream));
    return SS_OK;
}

// Reads the device status word (after the stream has been synchronized by
// the caller's copy) and, if it is set, clears it and fails.  The word is
// sticky: a condition raised by the last kernels of a call that returned
// without waiting is reported by the next check on the context.
ss_status status_failure(ss_ctx* c, uint32_t status, const std::string& where)
{
    (void)hipMemsetAsync((char*)c->info.p + offsetof(LevelInfo, status), 0, sizeof(uint32_t), c->stream);
    return fail(c, SS_EDEVICE, "device status " + std::to_string(status) + " " + where);
}

// Default light-bucket targets (percent of alpha) for hash and splitter buckets.
constexpr uint32_t kNlTargetHash = 50;
constexpr uint32_t kNlTargetLess = 35;

struct Params {
    uint32_t nl0, alpha, c, tmin, tmax, mode, tau;
    uint32_t tmax0, tmaxd;  // tile limits of the first and of the deeper levels
    bool auto_tiles;        // defaults apply: the first level's sample may choose smaller tiles
    uint32_t pool;          // records of the pool that replaces T below the first level (0: T)
    uint64_t seed;
};

ss_status resolve_params(ss_ctx* c, const ss_params* in, Params* p)
{
    ss_params d;
    ss_default_params(&d);
    const ss_params& s = in ? *in : d;
    p->nl0 = s.n_light_log2 ? s.n_light_log2 : d.n_light_log2;
    p->alpha = s.base_case ? s.base_case : d.base_case;
    p->c = s.sample_mult ? s.sample_mult : d.sample_mult;
    p->tmin = s.tile_min ? s.tile_min : d.tile_min;
    p->tmax = s.tile_max ? s.tile_max : 65536u;
    p->mode = s.hash_mode;
    p->tau = s.heavy_min;
    p->pool = s.temp_records;
    p->seed = s.seed;
    if (p->nl0 < 1 || p->nl0 > kLightBitsMax) return fail(c, SS_EINVAL, "n_light_log2 must be in [1, 10]");
    if (p->alpha < 64 || p->alpha > kAlphaMax) return fail(c, SS_EINVAL, "base_case must be in [64, 4096]");
    if (p->c < 1 || p->c > 4096) return fail(c, SS_EINVAL, "sample_mult must be in [1, 4096]");
    if (p->tau > kSampleMax) return fail(c, SS_EINVAL, "heavy_min must be at most 16384");
    auto pow2 = [](uint32_t x) { return x && !(x & (x - 1)); };
    if (!pow2(p->tmin) || !pow2(p->tmax) || p->tmin < 8192 || p->tmax > 65536 || p->tmin > p->tmax)
        return fail(c, SS_EINVAL, "tile_min/tile_max must be powers of two with 8192 <= tile_min <= tile_max <= 65536");
    if (p->mode > 1) return fail(c, SS_EINVAL, "hash_mode must be SS_HASH_MIX64 or SS_HASH_IDENTITY");
    p->auto_tiles = false;
    p->tmax0 = c && c->tile0 ? std::max(p->tmin, c->tile0) : p->tmax;
    p->tmaxd = c && c->tile_deep ? std::max(p->tmin, c->tile_deep) : p->tmax;
    return SS_OK;
}

// Subarray limits when the call leaves tile_max at 0: semisort_= uses at most
// 32768 records on the first level and 16384 below, semisort_< 32768 on the
// first level and 65536 below.  Shorter subarrays let neighbouring ones,
// distributed at the same time on one XCD, complete each other's partially
// written output lines in L2 (measured on 10^9 records against 65536
// throughout: semisort_= Zipf-1.2 3% and uniform keys 6% faster, semisort_<
// 2%); the reduction forms keep 65536, where heavy sums are added once per
// subarray and more subarrays cost more.
void default_tiles(const ss_ctx* c, const ss_params* in, Params* p, uint32_t first, uint32_t deeper)
{
    if (in && in->tile_max) return;
    if (!c->tile0) p->tmax0 = std::max(p->tmin, std::min(p->tmax, first));
    if (!c->tile_deep) p->tmaxd = std::max(p->tmin, std::min(p->tmax, deeper));
    p->auto_tiles = !c->tile0 && !c->tile_deep;
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes)
{
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + bbytes && y < x + abytes;
}

// ---------------------------------------------------------------- launches

// Base-case and copy jobs of one level: one launch per non-empty class.
// jobs holds kJobClasses lists of `cap` entries.
// Base-case and copy jobs of one level: one launch per non-empty class.
// jobs holds kJobClasses lists of `cap` entries.  MODE 0/1: semisort_= with
// the mixing / identity hash; MODE 2: semisort_<.
// Grid of a persistent base-case launch: the blocks that fit on the device
// at once (the occupancy of the kernel is queried once), at most one per job.
template <int MODE, typename V, int W, typename K = uint64_t>
uint32_t base_grid(const ss_ctx* c, uint32_t njobs)
{
    static const int per = [] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_base<MODE, V, W, K>, W * 64, 0) != hipSuccess || b < 1)
            b = 1;
        return b;
    }();
    return (uint32_t)std::min<uint64_t>(njobs, (uint64_t)per * (uint64_t)c->ncu);
}

template <int MODE, typename V, typename K>
void launch_jobs_m(ss_ctx* c, const uint32_t* njobs, uint32_t cap, const uint64_t* skw, const void* sv,
                   uint64_t* okw, void* ov)
{
    const K* sk = (const K*)skw;  // keys of K bytes
    K* ok = (K*)okw;
    const Job* jobs = (const Job*)c->jobs.p;
    LevelInfo* info = (LevelInfo*)c->info.p;
    const V* svv = (const V*)sv;
    V* ovv = (V*)ov;
    const Job* j1 = jobs + cap;
    const Job* j2 = jobs + 2 * (size_t)cap;
    const Job* j3 = jobs + 3 * (size_t)cap;
    if constexpr (MODE == 2) {
        if (njobs[0]) hipLaunchKernelGGL((k_base_less<V, 1, K>), dim3(njobs[0]), dim3(64), 0, c->stream, jobs, sk, svv, ok, ovv);
        if (njobs[1]) hipLaunchKernelGGL((k_base_less<V, 2, K>), dim3(njobs[1]), dim3(128), 0, c->stream, j1, sk, svv, ok, ovv);
        if (njobs[2]) hipLaunchKernelGGL((k_base_less<V, 4, K>), dim3(njobs[2]), dim3(256), 0, c->stream, j2, sk, svv, ok, ovv);
        if (njobs[3]) hipLaunchKernelGGL((k_base_less<V, 8, K>), dim3(njobs[3]), dim3(512), 0, c->stream, j3, sk, svv, ok, ovv);
    } else {
        uint64_t* sink = (uint64_t*)c->sink.p;
        if (njobs[0])
            hipLaunchKernelGGL((k_base<MODE, V, 1, K>), dim3(base_grid<MODE, V, 1, K>(c, njobs[0])), dim3(64), 0, c->stream,
                               jobs, njobs[0], sk, svv, ok, ovv, sink, info);
        if (njobs[1])
            hipLaunchKernelGGL((k_base<MODE, V, 2, K>), dim3(base_grid<MODE, V, 2, K>(c, njobs[1])), dim3(128), 0, c->stream,
                               j1, njobs[1], sk, svv, ok, ovv, sink, info);
        if (njobs[2])
            hipLaunchKernelGGL((k_base<MODE, V, 4, K>), dim3(base_grid<MODE, V, 4, K>(c, njobs[2])), dim3(256), 0, c->stream,
                               j2, njobs[2], sk, svv, ok, ovv, sink, info);
        if (njobs[3])
            hipLaunchKernelGGL((k_base_2pass<MODE, V, K>), dim3(njobs[3]), dim3(512), 0, c->stream, j3, sk, svv, ok, ovv,
                               info);
    }
    if (njobs[kCopyClass])
        hipLaunchKernelGGL((k_copy<V, K>), dim3(njobs[kCopyClass]), dim3(256), 0, c->stream,
                           jobs + (size_t)kCopyClass * cap, sk, svv, ok, ovv);
}

template <typename V, typename K = uint64_t>
void launch_jobs(ss_ctx* c, uint32_t mode, const uint32_t* njobs, uint32_t cap, const uint64_t* sk, const void* sv,
                 uint64_t* ok, void* ov, uint64_t records)
{
    ProfScope ps(c, SS_PROF_FINISH, records);
    if constexpr (!kWide<K>) {
        if (mode == 2) {
            launch_jobs_m<2, V, K>(c, njobs, cap, sk, sv, ok, ov);
            return;
        }
    }
    if (mode == 1) launch_jobs_m<1, V, K>(c, njobs, cap, sk, sv, ok, ov);
    else launch_jobs_m<0, V, K>(c, njobs, cap, sk, sv, ok, ov);
}

// part 0: the whole level; 1: sampling only; 2: everything after sampling;
// 3: sampling, counting and the prefix (no distribution); 4: counting and the
// prefix only; 5: the distribution only.
template <int MODE, typename V, typename K = uint64_t>
void launch_level(ss_ctx* c, const LevelArgs& a, uint32_t tiles, uint32_t chunks, uint64_t records, int part)
{
    const bool do_sample = part == 0 || part == 1 || part == 3;
    const bool do_count = part == 0 || part == 2 || part == 3 || part == 4;
    const bool do_dist = part == 0 || part == 2 || part == 5;
    if (do_sample) {
        ProfScope ps(c, SS_PROF_SAMPLE, a.nsegs);
        if constexpr (MODE == 2) hipLaunchKernelGGL((k_sample_less<K>), dim3(a.nsegs), dim3(1024), 0, c->stream, a);
        else hipLaunchKernelGGL((k_sample_heavy<MODE, K>), dim3(a.nsegs), dim3(1024), 0, c->stream, a);
    }
    if (do_count) {
        {
            ProfScope ps(c, SS_PROF_COUNT, records);
            if constexpr (MODE == 2) hipLaunchKernelGGL((k_count_less<K>), dim3(tiles), dim3(1024), 0, c->stream, a);
            else hipLaunchKernelGGL((k_count<MODE, K>), dim3(tiles), dim3(1024), 0, c->stream, a);
        }
        ProfScope ps(c, SS_PROF_SCAN, tiles);
        hipLaunchKernelGGL(k_scan_chunks, dim3(chunks), dim3(256), 0, c->stream, a);
        hipLaunchKernelGGL(k_scan_buckets, dim3(a.nsegs * kBucketGroups), dim3(1024), 0, c->stream, a);
        hipLaunchKernelGGL(k_scan_offsets, dim3(a.nsegs), dim3(1024), 0, c->stream, a);
        hipLaunchKernelGGL(k_scan_fill, dim3(chunks), dim3(256), 0, c->stream, a);
    }
    if (do_dist) {
        ProfScope ps(c, SS_PROF_DISTRIBUTE, records);
        if constexpr (kWide<K>) {
            // two registers per key: four records per thread keep the staged
            // sub-tile at the LDS size of the 64-bit form
            hipLaunchKernelGGL((k_distribute<V, 16, 4, 0, K>), dim3(tiles), dim3(1024), 0, c->stream, a);
        } else {
            switch (sizeof(K) == 8 ? c->dist_variant : std::min(c->dist_variant, 1)) {
            case 1:
                hipLaunchKernelGGL((k_distribute<V, 8, 8, 0, K>), dim3(tiles), dim3(512), 0, c->stream, a);
                break;
            case 2:
                hipLaunchKernelGGL((k_distribute_direct<V, 8, 8, 4>), dim3(tiles), dim3(512), 0, c->stream, a);
                break;
            case 3:
                hipLaunchKernelGGL((k_distribute_direct<V, 8, 8, 6>), dim3(tiles), dim3(512), 0, c->stream, a);
                break;
            case 4:
                hipLaunchKernelGGL((k_distribute_direct<V, 16, 8, 4>), dim3(tiles), dim3(1024), 0, c->stream, a);
                break;
            case 5:
                hipLaunchKernelGGL((k_distribute_direct<V, 4, 16, 6>), dim3(tiles), dim3(256), 0, c->stream, a);
                break;
            default:
                hipLaunchKernelGGL((k_distribute<V, 16, 8, 0, K>), dim3(tiles), dim3(1024), 0, c->stream, a);
            }
        }
    }
}

template <typename V, typename K = uint64_t>
void launch_level_v(ss_ctx* c, uint32_t mode, const LevelArgs& a, uint32_t tiles, uint32_t chunks,
                    uint64_t records, int part = 0)
{
    if constexpr (!kWide<K>) {
        if (mode == 2) {
            launch_level<2, V, K>(c, a, tiles, chunks, records, part);
            return;
        }
    }
    if (mode == 1) launch_level<1, V, K>(c, a, tiles, chunks, records, part);
    else launch_level<0, V, K>(c, a, tiles, chunks, records, part);
}

// Sizes a level needs: per-subproblem tables, counting matrix rows, chunk rows.
ss_status ensure_level(ss_ctx* c, uint32_t nsegs, uint32_t tiles, uint32_t chunks, bool wide = false)
{
    ss_status s;
    if (wide && (s = ensure(c, c->hrep, (size_t)nsegs * kHeavyMax * 16)) != SS_OK) return s;
    if ((s = ensure(c, c->C, (size_t)tiles * kNbStride * 4)) != SS_OK) return s;
    if ((s = ensure(c, c->P, (size_t)std::max(chunks, 1u) * kNbStride * 4)) != SS_OK) return s;
    if ((s = ensure(c, c->tot, (size_t)nsegs * kNbStride * 4)) != SS_OK) return s;
    if ((s = ensure(c, c->bstart, (size_t)nsegs * (kNbStride + 1) * 4)) != SS_OK) return s;
    if ((s = ensure(c, c->heavy_list, (size_t)nsegs * kHeavyMax * 8)) != SS_OK) return s;
    if ((s = ensure(c, c->tab_h, (size_t)nsegs * 2 * kHeavySlotsMax * 8)) != SS_OK) return s;
    if ((s = ensure(c, c->tab_id, (size_t)nsegs * 2 * kHeavySlotsMax * 2)) != SS_OK) return s;
    if ((s = ensure(c, c->bfin, (size_t)nsegs * kNbStride)) != SS_OK) return s;
    if ((s = ensure(c, c->bkey, (size_t)nsegs * kNbStride * 8)) != SS_OK) return s;
    if ((s = ensure(c, c->top, (size_t)nsegs * 4)) != SS_OK) return s;
    return SS_OK;
}

LevelArgs make_args(ss_ctx* c, const Params& p, uint32_t level, Seg* segs, uint32_t nsegs, uint32_t tile,
                    const uint64_t* sk, const void* sv, uint64_t* dk, void* dv, uint64_t* fk, void* fv)
{
    LevelArgs a;
    a.src_keys = sk;
    a.src_vals = sv;
    a.dst_keys = dk;
    a.dst_vals = dv;
    a.fin_keys = fk;
    a.fin_vals = fv;
    a.bids = (uint16_t*)c->bids.p;
    a.sink = (uint64_t*)c->sink.p;
    a.segs = segs;
    a.nsegs = nsegs;
    a.tile = tile;
    a.C = (uint32_t*)c->C.p;
    a.P = (uint32_t*)c->P.p;
    a.tot = (uint32_t*)c->tot.p;
    a.bstart = (uint32_t*)c->bstart.p;
    a.heavy_list = (uint64_t*)c->heavy_list.p;
    a.tab_h = (uint64_t*)c->tab_h.p;
    a.tab_id = (uint16_t*)c->tab_id.p;
    a.info = (LevelInfo*)c->info.p;
    a.seed = p.seed;
    a.level = level;
    a.sample_mult = p.c;
    a.heavy_min = p.tau;
    a.deep_div = c->deep_div;
    // Splitter buckets vary more in size than hash buckets (each splitter
    // interval holds a sampled share), so a smaller target keeps fewer of
    // them above alpha, where they would need one more level.
    a.nl_target = c->nl_target ? c->nl_target : (p.mode == 2 ? kNlTargetLess : kNlTargetHash);
    a.alpha = p.alpha;
    a.adaptive_nl = 1;
    a.ordered = p.mode == 2;
    a.bfin = (uint8_t*)c->bfin.p;
    a.bkey = (uint64_t*)c->bkey.p;
    a.hrep = (uint64_t*)c->hrep.p;
    a.top = (uint32_t*)c->top.p;
    a.fill_heavy = 0;
    a.reduce = 0;
    a.hsum = nullptr;
    a.res_keys = nullptr;
    a.res_vals = nullptr;
    a.rflag = nullptr;
    a.rop = 0;
    a.dims = nullptr;
    a.seg_cap = 0;
    a.q = nullptr;
    return a;
}

// Host-side prefix for the first level (same rule as k_seg_prefix).
void host_prefix(std::vector<Seg>& segs, const Params& p, uint32_t* tiles, uint32_t* chunks, uint32_t* tile)
{
    uint64_t total = 0;
    for (auto& s : segs) total += s.len;
    *tile = choose_tile(total, p.tmin, p.tmax0);
    uint32_t rt = 0, rc = 0;
    for (auto& s : segs) {
        s.ntiles = (s.len + *tile - 1) / *tile;
        s.tile0 = rt;
        s.chunk0 = rc;
        rt += s.ntiles;
        rc += (s.ntiles + kChunk - 1) / kChunk;
    }
    *tiles = rt;
    *chunks = rc;
}

// The second stream and its events, created on first use (default priority).
ss_status ensure_aux(ss_ctx* c)
{
    if (!c->aux) HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    for (hipEvent_t& e : c->fill_done)
        if (!e) HIP_OR_FAIL(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (hipEvent_t& e : c->fill_fork)
        if (!e) HIP_OR_FAIL(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return SS_OK;
}

ss_status ensure_jobs(ss_ctx* c, uint32_t per_class)
{
    if (per_class <= c->job_cap) return SS_OK;
    uint32_t want = std::max<uint32_t>(per_class, std::max<uint32_t>(4096, c->job_cap + c->job_cap / 2));
    ss_status r = ensure(c, c->jobs, (size_t)want * kJobClasses * sizeof(Job));
    if (r == SS_OK) c->job_cap = want;
    return r;
}

// Plans the next level from the buckets of the current one (subproblem list
// segs[cur] -> segs[cur ^ 1], job lists) and reads the level's counters back
// to the host; grows the lists and plans again when they overflow.
// With `between`, the plan is enqueued ahead of the level's distribution:
// between() launches the distribution after the plan's read-back, and the
// host waits for the read-back only (a retry waits for everything).
ss_status plan_level(ss_ctx* c, const Params& p, uint32_t level, uint32_t nsegs, int cur, uint32_t* seg_cap,
                     bool finals_in_out, bool reduce, bool fill, LevelInfo* out, uint32_t hash_bits = 64,
                     const std::function<void()>* between = nullptr)
{
    ss_status s;
    const int fb = level & 1;  // fill list of this level
    if (fill && c->fill_cap[fb] == 0) {
        if ((s = ensure(c, c->fills[fb], 4096 * sizeof(FillJob))) != SS_OK) return s;
        c->fill_cap[fb] = (uint32_t)(c->fills[fb].cap / sizeof(FillJob));
    }
    for (int attempt = 0;; ++attempt) {
        if (attempt && (s = reset_counters(c)) != SS_OK) return s;
        PlanArgs pa;
        pa.segs = (const Seg*)c->segs[cur].p;
        pa.nsegs = nsegs;
        pa.bstart = (const uint32_t*)c->bstart.p;
        pa.next = (Seg*)c->segs[cur ^ 1].p;
        pa.next_cap = *seg_cap;
        pa.jobs = (Job*)c->jobs.p;
        for (int k = 0; k < kJobClasses; ++k) {
            pa.job_base[k] = (uint64_t)k * c->job_cap;
            pa.job_capc[k] = c->job_cap;
        }
        pa.dims = nullptr;
        pa.cur_cap = 0;
        pa.info = (LevelInfo*)c->info.p;
        pa.alpha = p.alpha;
        pa.finals_in_out = finals_in_out;
        pa.ordered = p.mode == 2;
        pa.bfin = (const uint8_t*)c->bfin.p;
        pa.reduce = reduce;
        pa.fill = fill;
        pa.bkey = (const uint64_t*)c->bkey.p;
        pa.fills = (FillJob*)c->fills[fb].p;
        pa.fill_cap = c->fill_cap[fb];
        pa.hash_bits = hash_bits;
        {
            ProfScope ps(c, SS_PROF_PLAN, nsegs);
            hipLaunchKernelGGL(k_plan, dim3(nsegs), dim3(256), 0, c->stream, pa);
            hipLaunchKernelGGL(k_seg_prefix, dim3(1), dim3(1024), 0, c->stream, (Seg*)c->segs[cur ^ 1].p, *seg_cap,
                               (LevelInfo*)c->info.p, p.tmin, c->call_tmaxd ? c->call_tmaxd : p.tmaxd);
        }
        HIP_OR_FAIL(c, hipGetLastError());
        HIP_OR_FAIL(c, hipMemcpyAsync(c->info_host, c->info.p, sizeof(LevelInfo), hipMemcpyDeviceToHost, c->stream));
        if (between && attempt == 0) {
            if (!c->plan_ev) HIP_OR_FAIL(c, hipEventCreateWithFlags(&c->plan_ev, hipEventDisableTiming));
            HIP_OR_FAIL(c, hipEventRecord(c->plan_ev, c->stream));
            (*between)();
            HIP_OR_FAIL(c, hipGetLastError());
            HIP_OR_FAIL(c, hipEventSynchronize(c->plan_ev));
        } else {
            HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
        }
        const LevelInfo li = *c->info_host;
        if (li.status) {
            // the distribution enqueued by between() still writes the caller's
            // buffers: let it finish before reporting
            if (between) HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
            return status_failure(c, li.status, "at level " + std::to_string(level));
        }
        bool again = false;
        if (li.nsegs > *seg_cap) {
            // the current list must survive: copy it aside while both lists grow
            DevBuf keep;
            if ((s = ensure(c, keep, (size_t)nsegs * sizeof(Seg))) != SS_OK) return s;
            HIP_OR_FAIL(c, hipMemcpyAsync(keep.p, c->segs[cur].p, (size_t)nsegs * sizeof(Seg), hipMemcpyDeviceToDevice, c->stream));
            if ((s = ensure(c, c->segs[0], (size_t)li.nsegs * sizeof(Seg))) != SS_OK) return s;
            if ((s = ensure(c, c->segs[1], (size_t)li.nsegs * sizeof(Seg))) != SS_OK) return s;
            HIP_OR_FAIL(c, hipMemcpyAsync(c->segs[cur].p, keep.p, (size_t)nsegs * sizeof(Seg), hipMemcpyDeviceToDevice, c->stream));
            if ((s = release(c, keep)) != SS_OK) return s;
            *seg_cap = (uint32_t)std::min(c->segs[0].cap, c->segs[1].cap) / sizeof(Seg);
            again = true;
        }
        uint32_t jmax = 0;
        for (int k = 0; k < kJobClasses; ++k) jmax = std::max(jmax, li.njobs[k]);
        if (jmax > c->job_cap) {
            if ((s = ensure_jobs(c, jmax)) != SS_OK) return s;
            again = true;
        }
        if (li.nfills > c->fill_cap[fb]) {
            if (c->aux) HIP_OR_FAIL(c, hipStreamSynchronize(c->aux));  // a running fill may read the old list
            if ((s = ensure(c, c->fills[fb], (size_t)li.nfills * sizeof(FillJob))) != SS_OK) return s;
            c->fill_cap[fb] = (uint32_t)(c->fills[fb].cap / sizeof(FillJob));
            again = true;
        }
        if (again) continue;
        *out = li;
        return SS_OK;
    }
}

// The whole engine: `offs` are instance boundaries (host), total n = offs.back().
// Keys have K bytes (the key pointers are passed as uint64_t* and read as K).
template <typename V, typename K = uint64_t>
ss_status run_semisort(ss_ctx* c, const uint64_t* keys, const void* vals, const uint64_t* offs,
                             uint64_t ninst, uint64_t* keys_out, void* vals_out, const Params& p)
{
    const uint64_t n = offs[ninst];
    const bool inplace = keys_out == keys;
    // bounded temporary: the first level writes every bucket to the output,
    // the levels below refine groups of subproblems through a pool
    const bool pooled = p.pool != 0 && !inplace;
    c->call_tmaxd = 0;
    ss_status s;
    if ((s = stage_wait(c)) != SS_OK) return s;
    // first level: classify instances on the host
    c->host_segs.clear();
    for (auto& v : c->host_jobs) v.clear();
    uint64_t jrec = 0;
    for (uint64_t i = 0; i < ninst; ++i) {
        const uint32_t st = (uint32_t)offs[i];
        const uint32_t len = (uint32_t)(offs[i + 1] - offs[i]);
        if (len >= p.alpha) {
            Seg s{};
            s.start = st;
            s.len = len;
            s.ibase = st;
            s.nl_bits = (uint8_t)std::min(p.nl0, choose_nl(len, p.alpha, kLightBitsMax, 0));
            s.shift = 0;
            c->host_segs.push_back(s);
        } else if (len >= 2) {
            c->host_jobs[base_class(len)].push_back(Job{st, len});
            jrec += len;
        } else if (len == 1 && !inplace) {
            c->host_jobs[kCopyClass].push_back(Job{st, 1u});
            jrec += 1;
        }
    }
    uint32_t nsegs = (uint32_t)c->host_segs.size();
    uint32_t tiles = 0, chunks = 0, tile = p.tmin;
    uint64_t records = 0;
    for (const Seg& sg : c->host_segs) records += sg.len;
    if (nsegs) {
        host_prefix(c->host_segs, p, &tiles, &chunks, &tile);
        if (!pooled) {
            if ((s = ensure(c, c->t_keys, n * sizeof(K))) != SS_OK) return s;
            if ((s = ensure(c, c->t_vals, n * sizeof(V))) != SS_OK) return s;
        }
        if ((s = ensure(c, c->bids, n * 2)) != SS_OK) return s;
    }
    if ((s = ensure(c, c->info, sizeof(LevelInfo))) != SS_OK) return s;
    if ((s = ensure(c, c->sink, kSinkBytes)) != SS_OK) return s;
    uint32_t seg_cap = std::max<uint32_t>(nsegs, 1024);
    if ((s = ensure(c, c->segs[0], (size_t)seg_cap * sizeof(Seg))) != SS_OK) return s;
    if ((s = ensure(c, c->segs[1], (size_t)seg_cap * sizeof(Seg))) != SS_OK) return s;
    seg_cap = (uint32_t)std::min(c->segs[0].cap, c->segs[1].cap) / sizeof(Seg);
    uint32_t nj0[kJobClasses], nj0_max = 0, nj0_tot = 0;
    for (int k = 0; k < kJobClasses; ++k) {
        nj0[k] = (uint32_t)c->host_jobs[k].size();
        nj0_max = std::max(nj0_max, nj0[k]);
        nj0_tot += nj0[k];
    }
    if ((s = ensure_jobs(c, std::max<uint32_t>(nj0_max, 4096))) != SS_OK) return s;

    if ((s = reset_counters(c)) != SS_OK) return s;
    if (nj0_tot) {
        if ((s = ensure_pinned(c, (void**)&c->job_stage, &c->job_stage_cap, (size_t)nj0_tot * sizeof(Job))) != SS_OK)
            return s;
        size_t o = 0;
        for (int k = 0; k < kJobClasses; ++k) {
            if (!nj0[k]) continue;
            memcpy(c->job_stage + o, c->host_jobs[k].data(), nj0[k] * sizeof(Job));
            HIP_OR_FAIL(c, hipMemcpyAsync((Job*)c->jobs.p + (size_t)k * c->job_cap, c->job_stage + o,
                                          nj0[k] * sizeof(Job), hipMemcpyHostToDevice, c->stream));
            o += nj0[k];
        }
        launch_jobs<V, K>(c, p.mode, nj0, c->job_cap, keys, vals, keys_out, vals_out, jrec);
        HIP_OR_FAIL(c, hipGetLastError());
    }
    if (!nsegs) {
        // wait: the next call reuses the pinned job staging buffer
        if (nj0_tot) {
            HIP_OR_FAIL(c, hipMemcpyAsync(c->info_host, c->info.p, sizeof(LevelInfo), hipMemcpyDeviceToHost, c->stream));
            HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
            if (c->info_host->status) return status_failure(c, c->info_host->status, "in the base cases");
        }
        return SS_OK;
    }
    if ((s = ensure_pinned(c, (void**)&c->seg_stage, &c->seg_stage_cap, nsegs * sizeof(Seg))) != SS_OK) return s;
    memcpy(c->seg_stage, c->host_segs.data(), nsegs * sizeof(Seg));
    int cur = 0;
    HIP_OR_FAIL(c, hipMemcpyAsync(c->segs[cur].p, c->seg_stage, nsegs * sizeof(Seg), hipMemcpyHostToDevice, c->stream));

    // Where the current level's records are; T is the temporary array, or
    // the pool placed so that the current group's positions index it.
    enum Where { kInput, kOut, kTemp };
    // in place, the caller's input is the output: the first level must not
    // write final buckets there while other blocks still read it
    Where loc = inplace ? kOut : kInput;
    uint64_t* T_k = (uint64_t*)c->t_keys.p;
    void* T_v = c->t_vals.p;
    auto kptr = [&](Where w) -> uint64_t* { return w == kInput ? (uint64_t*)keys : w == kOut ? keys_out : T_k; };
    auto vptr = [&](Where w) -> void* { return w == kInput ? (void*)vals : w == kOut ? vals_out : T_v; };
    bool fill_used[2] = {false, false};
    // on an early error return, do not leave a fill running into the caller's buffers
    struct AuxGuard {
        ss_ctx* c;
        bool armed = false;
        ~AuxGuard()
        {
            if (armed && c->aux) (void)hipStreamSynchronize(c->aux);
        }
    } guard{c};
    // One level over the current subproblem list (segs[cur]); all_to_out:
    // every bucket goes to the output (the first level of the pooled form).
    auto step = [&](uint32_t level, bool all_to_out) -> ss_status {
        ss_status s;
        // Buckets that need more work go to the buffer that is not the
        // source; final buckets go straight to the output unless the output
        // is the source (other blocks still read it).
        Where dst, fin;
        if (all_to_out) dst = fin = kOut;
        else if (loc == kOut) dst = fin = kTemp;
        else if (loc == kTemp) dst = fin = kOut;
        else {  // the caller's input, distinct from the output
            dst = kTemp;
            fin = kOut;
        }
        uint64_t* dst_k = kptr(dst);
        void* dst_v = vptr(dst);
        if ((s = ensure_level(c, nsegs, tiles, chunks, kWide<K>)) != SS_OK) return s;
        if ((s = reset_counters(c)) != SS_OK) return s;
        LevelArgs a = make_args(c, p, level, (Seg*)c->segs[cur].p, nsegs, tile, kptr(loc), vptr(loc), dst_k, dst_v,
                                kptr(fin), vptr(fin));
        // one-key buckets written to the output: only their values move,
        // their keys are filled as constant runs on the second stream while
        // the next level runs (the two touch disjoint ranges).  128-bit keys
        // move with their values.
        const bool fill = !kWide<K> && fin == kOut;
        const int fb = level & 1;
        a.fill_heavy = fill;
        // semisort_<: the level is planned before its distribution, so that
        // its key fills run beside the distribution instead of beside the
        // next level's base cases (10^9 records: exponential keys 2.2-2.5%
        // faster, Zipf-0.8 unchanged).  semisort_= keeps the fills after the
        // distribution: beside it they slow the first level more than they
        // save (Zipf-1.2 1.7% slower).  The fills write only the keys of
        // one-key buckets, which the distribution does not write.
        const bool early = fill && p.mode == 2;
        // Below 2 * 2048 * tile_min records every level already takes
        // tile_min-record subarrays (about 2048 subarrays per level), so the
        // sample's count could change nothing: no synchronization for it.
        const bool tiles_open = (uint64_t)records / 2048 >= 2ull * p.tmin;
        if (level == 0 && p.auto_tiles && nsegs == 1 && p.mode != 2 && tiles_open) {
            // Light-dominated input (under half of the first level's sample on
            // heavy keys): subarrays of 8192 records on every level, so that
            // neighbouring ones complete each other's partial lines in L2
            // (uniform keys at 10^9: 7% faster; heavy-dominated inputs lose
            // with them).  One synchronization reads the sample's count.
            launch_level_v<V, K>(c, p.mode, a, tiles, chunks, records, 1);
            HIP_OR_FAIL(c, hipGetLastError());
            HIP_OR_FAIL(c, hipMemcpyAsync(c->info_host, c->info.p, sizeof(LevelInfo), hipMemcpyDeviceToHost,
                                          c->stream));
            HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
            const LevelInfo si = *c->info_host;
            if (si.status) return status_failure(c, si.status, "at level 0 sampling");
            const uint32_t small = std::max(p.tmin, 8192u);
            if (si.smp_total && 2ull * si.smp_heavy < si.smp_total && small < tile) {
                c->call_tmaxd = small;
                tile = small;
                c->seg_stage[0].ntiles = (uint32_t)((c->seg_stage[0].len + (uint64_t)tile - 1) / tile);
                tiles = c->seg_stage[0].ntiles;
                chunks = (tiles + kChunk - 1) / kChunk;
                HIP_OR_FAIL(c, hipMemcpyAsync((char*)c->segs[cur].p + offsetof(Seg, ntiles), &c->seg_stage[0].ntiles,
                                              sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
                // more subarrays: a larger counting matrix and chunk table; the
                // buffers the sampling kernel filled keep their size.  The
                // level's arguments take the (possibly reallocated) pointers.
                if ((s = ensure(c, c->C, (size_t)tiles * kNbStride * 4)) != SS_OK) return s;
                if ((s = ensure(c, c->P, (size_t)std::max(chunks, 1u) * kNbStride * 4)) != SS_OK) return s;
                a.C = (uint32_t*)c->C.p;
                a.P = (uint32_t*)c->P.p;
                a.tile = tile;
            }
            launch_level_v<V, K>(c, p.mode, a, tiles, chunks, records, early ? 4 : 2);
        } else {
            launch_level_v<V, K>(c, p.mode, a, tiles, chunks, records, early ? 3 : 0);
        }
        HIP_OR_FAIL(c, hipGetLastError());
        if (fill_used[fb]) HIP_OR_FAIL(c, hipStreamWaitEvent(c->stream, c->fill_done[fb], 0));  // list reuse

        LevelInfo li;
        const std::function<void()> dist = [&] { launch_level_v<V, K>(c, p.mode, a, tiles, chunks, records, 5); };
        if ((s = plan_level(c, p, level, nsegs, cur, &seg_cap, fin == kOut, false, fill, &li,
                            KeyTraits<K>::hash_bits, early ? &dist : nullptr)) != SS_OK)
            return s;
        if constexpr (!kWide<K>) if (li.nfills) {
            if ((s = ensure_aux(c)) != SS_OK) return s;
            {
                ProfScope ps(c, SS_PROF_FILL, li.fill_records, c->aux);
                hipLaunchKernelGGL((k_fill<K>), dim3(li.nfills), dim3(1024), 0, c->aux, (const FillJob*)c->fills[fb].p,
                                   (K*)keys_out);
            }
            HIP_OR_FAIL(c, hipEventRecord(c->fill_done[fb], c->aux));
            fill_used[fb] = true;
            guard.armed = true;
        }
        launch_jobs<V, K>(c, p.mode, li.njobs, c->job_cap, dst_k, dst_v, keys_out, vals_out, li.job_records);
        HIP_OR_FAIL(c, hipGetLastError());
        nsegs = li.nsegs;
        records = li.records;
        tiles = li.tiles;
        chunks = li.chunks;
        tile = li.tile;
        loc = dst;
        cur ^= 1;
        return SS_OK;
    };
    uint32_t level = 0;
    if (!pooled) {
        while (nsegs)
            if ((s = step(level++, false)) != SS_OK) return s;
    } else {
        if ((s = step(level++, true)) != SS_OK) return s;
        if (nsegs) {
            // the subproblems below the first level, on the host, in ascending
            // positions (the planning step lists each subproblem's buckets
            // thread by thread)
            const uint32_t nall = nsegs;
            if ((s = ensure_pinned(c, (void**)&c->seg_stage, &c->seg_stage_cap, (size_t)nall * sizeof(Seg))) != SS_OK)
                return s;
            HIP_OR_FAIL(c, hipMemcpyAsync(c->seg_stage, c->segs[cur].p, (size_t)nall * sizeof(Seg),
                                          hipMemcpyDeviceToHost, c->stream));
            HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
            std::vector<Seg> all(c->seg_stage, c->seg_stage + nall);
            std::sort(all.begin(), all.end(), [](const Seg& x, const Seg& y) { return x.start < y.start; });
            // groups of consecutive subproblems spanning at most `cap`
            // positions, cap = the pool size, or the longest subproblem
            uint64_t cap = p.pool;
            for (const Seg& sg : all) cap = std::max<uint64_t>(cap, sg.len);
            cap = std::min<uint64_t>(cap, n);
            if ((s = ensure(c, c->t_keys, cap * sizeof(K))) != SS_OK) return s;
            if ((s = ensure(c, c->t_vals, cap * sizeof(V))) != SS_OK) return s;
            const uint32_t tile1 = tile;
            for (uint32_t i0 = 0; i0 < nall;) {
                const uint64_t g0 = all[i0].start;
                uint32_t i1 = i0 + 1;
                while (i1 < nall && (uint64_t)all[i1].start + all[i1].len - g0 <= cap) ++i1;
                // the group's subarrays numbered from 0 (same subarray size)
                uint32_t gt = 0, gc = 0;
                uint64_t grec = 0;
                for (uint32_t j = i0; j < i1; ++j) {
                    Seg sg = all[j];
                    sg.tile0 = gt;
                    sg.chunk0 = gc;
                    gt += sg.ntiles;
                    gc += (sg.ntiles + kChunk - 1) / kChunk;
                    grec += sg.len;
                    c->seg_stage[j - i0] = sg;
                }
                nsegs = i1 - i0;
                if ((s = ensure(c, c->segs[cur], (size_t)std::max(nsegs, seg_cap) * sizeof(Seg))) != SS_OK) return s;
                HIP_OR_FAIL(c, hipMemcpyAsync(c->segs[cur].p, c->seg_stage, (size_t)nsegs * sizeof(Seg),
                                              hipMemcpyHostToDevice, c->stream));
                tiles = gt;
                chunks = gc;
                records = grec;
                tile = tile1;
                // the pool stands for positions [g0, g0 + cap): its address
                // less g0 records, so that the kernels' absolute positions
                // land in it (formed as an integer: only positions of the
                // group are ever added back)
                T_k = (uint64_t*)((uintptr_t)c->t_keys.p - (uintptr_t)g0 * sizeof(K));
                T_v = (void*)((uintptr_t)c->t_vals.p - (uintptr_t)g0 * sizeof(V));
                loc = kOut;
                for (uint32_t lv = level; nsegs; ++lv)
                    if ((s = step(lv, false)) != SS_OK) return s;
                i0 = i1;
            }
        }
    }
    // The last level's base cases and fills are left running: the call
    // returns once they are enqueued (the stream waits for the fills), and a
    // range error they raise is reported by the next check of the status word
    // (ss_sync or the next call).
    for (int b = 0; b < 2; ++b)
        if (fill_used[b]) HIP_OR_FAIL(c, hipStreamWaitEvent(c->stream, c->fill_done[b], 0));
    guard.armed = false;
    return SS_OK;
}

// ---------------------------------------------------------------- device-sized batches

// Resident grid of a device-sized kernel: as many blocks as fit on the device
// at once (occupancy queried once per kernel), at most `bound`.
template <auto K>
uint32_t ds_grid(const ss_ctx* c, int threads, uint64_t bound)
{
    static const int per = [threads] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, K, threads, 0) != hipSuccess || b < 1) b = 1;
        return b;
    }();
    const uint64_t g = std::min<uint64_t>(bound, (uint64_t)per * (uint64_t)c->ncu);
    return (uint32_t)std::max<uint64_t>(g, 1);
}

// The same for kernels with per-XCD work queues: a multiple of 8 blocks.
template <auto K>
uint32_t ds_grid_xcd(const ss_ctx* c, int threads)
{
    return (ds_grid<K>(c, threads, ~0ull) + 7u) & ~7u;
}

// Grows a buffer outside stream capture only: a captured call must find its
// workspace already sized by an earlier uncaptured call.
ss_status ensure_ds(ss_ctx* c, DevBuf& b, size_t bytes, bool capturing)
{
    if (bytes <= b.cap) return SS_OK;
    if (capturing)
        return fail(c, SS_EINVAL, "the workspace must grow, which stream capture does not allow: make one "
                                  "uncaptured call with the same sizes first");
    return ensure(c, b, bytes);
}

// Work-queue counters per device-sized level: [0, 8) counting and [8, 16)
// distribution (per XCD), 16 the two-pass base cases of the level's jobs.
constexpr uint32_t kQueueWords = 32;

// Upper bounds of one device-sized level over n records: subproblems hold at
// least alpha records (the first level's at most one per instance), so
// nsegs <= n / alpha; a level of R <= n records in nsegs subproblems has at
// most R / tile + nsegs subarrays; a job of class c holds at least
// 2, 513, 1025, 2049 records, and copy jobs at least one.
struct DsBounds {
    uint64_t segs, tiles, chunks;
    uint64_t jobs[kJobClasses];
};

DsBounds ds_bounds(uint64_t n, uint64_t nseg, const Params& p)
{
    DsBounds b;
    b.segs = std::max<uint64_t>(std::min<uint64_t>(nseg, n / p.alpha), n / p.alpha) + 1;
    b.tiles = n / p.tmin + b.segs;
    b.chunks = b.tiles / kChunk + b.segs;
    b.jobs[0] = n / 2 + 1;
    b.jobs[1] = n / 513 + 1;
    b.jobs[2] = n / 1025 + 1;
    b.jobs[3] = n / 2049 + 1;
    b.jobs[kCopyClass] = n + n / kCopyChunk + 1;
    return b;
}

// Workspace of a device-sized batch: every buffer the levels use, taken
// either from the context's growable buffers or, for the call that must not
// allocate, carved out of the library's static scratch array.
enum DsBufId {
    kDsTKeys, kDsTVals, kDsBids, kDsSink, kDsInfos, kDsJobs, kDsQueues, kDsSegs0, kDsSegs1, kDsC, kDsP, kDsTot,
    kDsBstart, kDsHeavy, kDsTabH, kDsTabId, kDsBfin, kDsBkey, kDsTop, kDsFills0, kDsFills1, kDsBufCount
};

struct DsSpace {
    void* p[kDsBufCount];
    uint32_t fill_cap;  // entries of each key-fill list
};

// Bytes of every buffer for a batch of n records in ninst instances.
void ds_sizes(uint64_t n, uint32_t vb, const DsBounds& b, uint32_t levels, uint64_t jtot, uint64_t fcap,
              size_t (&sz)[kDsBufCount])
{
    sz[kDsTKeys] = n * 8;
    sz[kDsTVals] = n * vb;
    sz[kDsBids] = n * 2;
    sz[kDsSink] = 512;
    sz[kDsInfos] = (size_t)(levels + 1) * sizeof(LevelInfo);
    sz[kDsJobs] = jtot * sizeof(Job);
    sz[kDsQueues] = (size_t)(levels + 1) * kQueueWords * 4;
    sz[kDsSegs0] = sz[kDsSegs1] = b.segs * sizeof(Seg);
    sz[kDsC] = b.tiles * kNbStride * 4;
    sz[kDsP] = b.chunks * kNbStride * 4;
    sz[kDsTot] = b.segs * kNbStride * 4;
    sz[kDsBstart] = b.segs * (kNbStride + 1) * 4;
    sz[kDsHeavy] = b.segs * kHeavyMax * 8;
    sz[kDsTabH] = b.segs * 2 * kHeavySlotsMax * 8;
    sz[kDsTabId] = b.segs * 2 * kHeavySlotsMax * 2;
    sz[kDsBfin] = b.segs * kNbStride;
    sz[kDsBkey] = b.segs * kNbStride * 8;
    sz[kDsTop] = b.segs * 4;
    sz[kDsFills0] = sz[kDsFills1] = fcap * sizeof(FillJob);
}

// The context's buffers, grown outside capture only.
ss_status ds_space_ctx(ss_ctx* c, const size_t (&sz)[kDsBufCount], bool capturing, DsSpace* sp)
{
    DevBuf* bufs[kDsBufCount] = {&c->t_keys, &c->t_vals, &c->bids, &c->sink, &c->ds_info, &c->ds_jobs, &c->ds_q,
                                 &c->segs[0], &c->segs[1], &c->C, &c->P, &c->tot, &c->bstart, &c->heavy_list,
                                 &c->tab_h, &c->tab_id, &c->bfin, &c->bkey, &c->top, &c->fills[0], &c->fills[1]};
    ss_status s;
    for (int i = 0; i < kDsBufCount; ++i) {
        if ((s = ensure_ds(c, *bufs[i], sz[i], capturing)) != SS_OK) return s;
        sp->p[i] = bufs[i]->p;
    }
    for (int k = 0; k < 2; ++k)
        c->fill_cap[k] = (uint32_t)std::min<uint64_t>(c->fills[k].cap / sizeof(FillJob), 0xFFFFFFFFu);
    sp->fill_cap = std::min(c->fill_cap[0], c->fill_cap[1]);
    return SS_OK;
}

// Consecutive 256-byte aligned pieces of [base, base + cap); the bytes
// needed, whether or not they fit, in *need.
bool ds_space_carve(void* base, size_t cap, const size_t (&sz)[kDsBufCount], uint64_t fcap, DsSpace* sp,
                    size_t* need)
{
    size_t o = 0;
    for (int i = 0; i < kDsBufCount; ++i) {
        sp->p[i] = (char*)base + o;
        o += (sz[i] + 255) & ~(size_t)255;
    }
    sp->fill_cap = (uint32_t)std::min<uint64_t>(fcap, 0xFFFFFFFFu);
    *need = o;
    return o <= cap;
}

LevelArgs make_args_ds(ss_ctx* c, const DsSpace& sp, const Params& p, uint32_t level, Seg* segs,
                       const uint64_t* sk, const void* sv, uint64_t* dk, void* dv, uint64_t* fk, void* fv)
{
    LevelArgs a = make_args(c, p, level, segs, 0, 0, sk, sv, dk, dv, fk, fv);
    a.bids = (uint16_t*)sp.p[kDsBids];
    a.sink = (uint64_t*)sp.p[kDsSink];
    a.C = (uint32_t*)sp.p[kDsC];
    a.P = (uint32_t*)sp.p[kDsP];
    a.tot = (uint32_t*)sp.p[kDsTot];
    a.bstart = (uint32_t*)sp.p[kDsBstart];
    a.heavy_list = (uint64_t*)sp.p[kDsHeavy];
    a.tab_h = (uint64_t*)sp.p[kDsTabH];
    a.tab_id = (uint16_t*)sp.p[kDsTabId];
    a.bfin = (uint8_t*)sp.p[kDsBfin];
    a.bkey = (uint64_t*)sp.p[kDsBkey];
    a.top = (uint32_t*)sp.p[kDsTop];
    return a;
}

template <int MODE, typename V>
void launch_jobs_ds(ss_ctx* c, const JobLists& jl, const LevelInfo* dims, uint32_t* q, const uint64_t* sk,
                    const void* sv, uint64_t* ok, void* ov, LevelInfo* info, uint64_t* sink)
{
    const V* svv = (const V*)sv;
    V* ovv = (V*)ov;
    const uint32_t* cnt = dims->njobs;
    hipLaunchKernelGGL((k_base_ds<MODE, V, 1>), dim3(ds_grid<k_base_ds<MODE, V, 1>>(c, 64, jl.cap[0])), dim3(64), 0,
                       c->stream, jl.jobs + jl.base[0], cnt + 0, jl.cap[0], sk, svv, ok, ovv, sink, info);
    hipLaunchKernelGGL((k_base_ds<MODE, V, 2>), dim3(ds_grid<k_base_ds<MODE, V, 2>>(c, 128, jl.cap[1])), dim3(128), 0,
                       c->stream, jl.jobs + jl.base[1], cnt + 1, jl.cap[1], sk, svv, ok, ovv, sink, info);
    hipLaunchKernelGGL((k_base_ds<MODE, V, 4>), dim3(ds_grid<k_base_ds<MODE, V, 4>>(c, 256, jl.cap[2])), dim3(256), 0,
                       c->stream, jl.jobs + jl.base[2], cnt + 2, jl.cap[2], sk, svv, ok, ovv, sink, info);
    hipLaunchKernelGGL((k_base_2pass_ds<MODE, V>), dim3(ds_grid<k_base_2pass_ds<MODE, V>>(c, 512, jl.cap[3])),
                       dim3(512), 0, c->stream, jl.jobs + jl.base[3], cnt + 3, jl.cap[3], q + 16, sk, svv, ok, ovv,
                       info);
    hipLaunchKernelGGL((k_copy_ds<V>), dim3(ds_grid<k_copy_ds<V>>(c, 256, jl.cap[kCopyClass])), dim3(256), 0,
                       c->stream, jl.jobs + jl.base[kCopyClass], cnt + kCopyClass, jl.cap[kCopyClass], sk, svv, ok,
                       ovv);
}

template <int MODE, typename V>
void launch_level_ds(ss_ctx* c, const LevelArgs& a, const DsBounds& b)
{
    hipLaunchKernelGGL((k_sample_heavy_ds<MODE>), dim3(ds_grid<k_sample_heavy_ds<MODE>>(c, 1024, b.segs)), dim3(1024),
                       0, c->stream, a);
    hipLaunchKernelGGL((k_count_ds<MODE>), dim3(ds_grid_xcd<k_count_ds<MODE>>(c, 1024)), dim3(1024), 0, c->stream,
                       a);
    hipLaunchKernelGGL(k_scan_chunks_ds, dim3(ds_grid<k_scan_chunks_ds>(c, 256, b.chunks)), dim3(256), 0, c->stream,
                       a);
    hipLaunchKernelGGL(k_scan_buckets_ds, dim3(ds_grid<k_scan_buckets_ds>(c, 1024, b.segs * kBucketGroups)),
                       dim3(1024), 0, c->stream, a);
    hipLaunchKernelGGL(k_scan_offsets_ds, dim3(ds_grid<k_scan_offsets_ds>(c, 1024, b.segs)), dim3(1024), 0,
                       c->stream, a);
    hipLaunchKernelGGL(k_scan_fill_ds, dim3(ds_grid<k_scan_fill_ds>(c, 256, b.chunks)), dim3(256), 0, c->stream, a);
    hipLaunchKernelGGL((k_distribute_ds<V, 16, 8, 0>), dim3(ds_grid_xcd<k_distribute_ds<V, 16, 8, 0>>(c, 1024)),
                       dim3(1024), 0, c->stream, a);
}

// Bounds, job-list layout and key-fill list size of a device-sized batch.
struct DsPlan {
    DsBounds b;
    JobLists jl;
    uint64_t jtot, fcap;
};

ss_status ds_plan(ss_ctx* c, uint64_t n, uint64_t ninst, const Params& p, DsPlan* d)
{
    d->b = ds_bounds(n, ninst, p);
    if (d->b.segs >= (1ull << 31) || d->b.tiles >= (1ull << 31) || d->b.jobs[kCopyClass] >= (1ull << 32))
        return fail(c, SS_EINVAL, "batch too large for the device-sized form");
    d->jtot = 0;
    for (int k = 0; k < kJobClasses; ++k) {
        d->jl.base[k] = d->jtot;
        d->jl.cap[k] = (uint32_t)d->b.jobs[k];
        d->jtot += d->b.jobs[k];
    }
    // key-fill lists of one-key buckets (alternating levels), run on the
    // second stream as in the host-sized engine: at most one job per
    // non-empty heavy bucket plus one per kFillChunk records
    d->fcap = std::min<uint64_t>(d->b.segs * kHeavyMax, n) + n / kFillChunk + 1;
    return SS_OK;
}

// The batch with every level sized on the device: no host synchronization
// and no allocation (the workspace `sp` is sized already), so the whole call
// can be captured into a graph.  `offs` is a device array of ninst + 1
// offsets.
template <int MODE, typename V>
ss_status run_semisort_ds(ss_ctx* c, const uint64_t* keys, const void* vals, const uint64_t* offs, uint64_t ninst,
                          uint64_t n, uint64_t* keys_out, void* vals_out, const Params& p, uint32_t levels,
                          const DsPlan& d, const DsSpace& sp)
{
    const bool inplace = keys_out == keys;
    const DsBounds& b = d.b;
    JobLists jl = d.jl;
    jl.jobs = (Job*)sp.p[kDsJobs];
    bool fill_used[2] = {false, false};
    const uint32_t seg_cap = (uint32_t)b.segs;
    LevelInfo* infos = (LevelInfo*)sp.p[kDsInfos];
    uint64_t* sink = (uint64_t*)sp.p[kDsSink];
    Seg* segs[2] = {(Seg*)sp.p[kDsSegs0], (Seg*)sp.p[kDsSegs1]};
    FillJob* fills[2] = {(FillJob*)sp.p[kDsFills0], (FillJob*)sp.p[kDsFills1]};

    // counts of every level start at zero; so does the call's status word
    const uint32_t iw = (uint32_t)((levels + 1) * sizeof(LevelInfo) / 4);
    hipLaunchKernelGGL(k_ds_clear, dim3((iw + 255) / 256), dim3(256), 0, c->stream, (uint32_t*)infos, iw);
    uint32_t* qs = (uint32_t*)sp.p[kDsQueues];  // per level: kQueueWords counters
    hipLaunchKernelGGL(k_ds_clear, dim3(((levels + 1) * kQueueWords + 255) / 256), dim3(256), 0, c->stream, qs,
                       (levels + 1) * kQueueWords);
    hipLaunchKernelGGL(k_ds_clear, dim3(1), dim3(256), 0, c->stream, (uint32_t*)c->info.p,
                       (uint32_t)(sizeof(LevelInfo) / 4));
    hipLaunchKernelGGL(k_ds_check_offsets, dim3((uint32_t)std::min<uint64_t>((ninst + 255) / 256, 4096)),
                       dim3(256), 0, c->stream, offs, (uint32_t)ninst, n, infos);
    hipLaunchKernelGGL(k_ds_plan_instances, dim3((uint32_t)std::min<uint64_t>((ninst + 255) / 256, 4096)), dim3(256),
                       0, c->stream, offs, (uint32_t)ninst, n, p.alpha, p.nl0, (uint32_t)inplace,
                       segs[0], seg_cap, jl, infos);
    hipLaunchKernelGGL(k_seg_prefix, dim3(1), dim3(1024), 0, c->stream, segs[0], seg_cap, infos, p.tmin,
                       p.tmax0);
    launch_jobs_ds<MODE, V>(c, jl, infos, qs, keys, vals, keys_out, vals_out, infos, sink);
    HIP_OR_FAIL(c, hipGetLastError());

    const uint64_t* loc_k = keys;
    const void* loc_v = vals;
    uint64_t* T_k = (uint64_t*)sp.p[kDsTKeys];
    void* T_v = sp.p[kDsTVals];
    int cur = 0;
    for (uint32_t level = 0; level < levels; ++level) {
        // buffers as in the host-sized engine (the sequence does not depend on the data)
        uint64_t* dst_k;
        void* dst_v;
        uint64_t* fin_k;
        void* fin_v;
        if (loc_k == keys_out) {
            dst_k = fin_k = T_k;
            dst_v = fin_v = T_v;
        } else if (loc_k == T_k) {
            dst_k = fin_k = keys_out;
            dst_v = fin_v = vals_out;
        } else {
            dst_k = T_k;
            dst_v = T_v;
            fin_k = keys_out;
            fin_v = vals_out;
        }
        LevelArgs a = make_args_ds(c, sp, p, level, segs[cur], loc_k, loc_v, dst_k, dst_v, fin_k, fin_v);
        a.dims = infos + level;
        a.seg_cap = seg_cap;
        a.info = infos + level + 1;
        // one-key buckets bound for keys_out move only their values; their
        // keys are filled on the second stream while the next level runs
        const bool fill = fin_k == keys_out;
        const int fb = level & 1;
        a.fill_heavy = fill;
        a.q = qs + (size_t)(level + 1) * kQueueWords;
        launch_level_ds<MODE, V>(c, a, b);
        if (fill_used[fb]) HIP_OR_FAIL(c, hipStreamWaitEvent(c->stream, c->fill_done[fb], 0));  // list reuse

        PlanArgs pa;
        pa.segs = segs[cur];
        pa.nsegs = 0;
        pa.bstart = a.bstart;
        pa.next = segs[cur ^ 1];
        pa.next_cap = seg_cap;
        pa.jobs = jl.jobs;
        for (int k = 0; k < kJobClasses; ++k) {
            pa.job_base[k] = jl.base[k];
            pa.job_capc[k] = jl.cap[k];
        }
        pa.info = infos + level + 1;
        pa.alpha = p.alpha;
        pa.finals_in_out = fin_k == keys_out;
        pa.ordered = 0;
        pa.bfin = a.bfin;
        pa.reduce = 0;
        pa.fill = fill;
        pa.bkey = a.bkey;
        pa.fills = fills[fb];
        pa.fill_cap = sp.fill_cap;
        pa.dims = infos + level;
        pa.cur_cap = seg_cap;
        hipLaunchKernelGGL(k_plan_ds, dim3(ds_grid<k_plan_ds>(c, 256, b.segs)), dim3(256), 0, c->stream, pa);
        hipLaunchKernelGGL(k_seg_prefix, dim3(1), dim3(1024), 0, c->stream, segs[cur ^ 1], seg_cap,
                           infos + level + 1, p.tmin, p.tmaxd);
        if (fill) {
            HIP_OR_FAIL(c, hipEventRecord(c->fill_fork[fb], c->stream));
            HIP_OR_FAIL(c, hipStreamWaitEvent(c->aux, c->fill_fork[fb], 0));
            // one block per CU: the fill is bound by HBM writes and leaves
            // room for the base cases running beside it
            hipLaunchKernelGGL(k_fill_ds, dim3((uint32_t)std::min<uint64_t>(d.fcap, (uint64_t)c->ncu)), dim3(1024),
                               0, c->aux, (const FillJob*)fills[fb], &infos[level + 1].nfills, sp.fill_cap, keys_out);
            HIP_OR_FAIL(c, hipEventRecord(c->fill_done[fb], c->aux));
            fill_used[fb] = true;
        }
        launch_jobs_ds<MODE, V>(c, jl, infos + level + 1, qs + (size_t)(level + 1) * kQueueWords, dst_k, dst_v,
                                keys_out, vals_out, infos + level + 1, sink);
        HIP_OR_FAIL(c, hipGetLastError());
        loc_k = dst_k;
        loc_v = dst_v;
        cur ^= 1;
    }
    for (int k = 0; k < 2; ++k)  // joins the second stream (also ends its part of a capture)
        if (fill_used[k]) HIP_OR_FAIL(c, hipStreamWaitEvent(c->stream, c->fill_done[k], 0));
    hipLaunchKernelGGL(k_ds_finish, dim3(1), dim3(64), 0, c->stream, (const LevelInfo*)infos, levels, seg_cap, jl,
                       sp.fill_cap, (LevelInfo*)c->info.p);
    HIP_OR_FAIL(c, hipGetLastError());
    return SS_OK;
}

// The device-sized batch on the context's own workspace, grown (outside
// capture) to the call's worst case.
template <int MODE, typename V>
ss_status run_semisort_ds_ctx(ss_ctx* c, const uint64_t* keys, const void* vals, const uint64_t* offs,
                              uint64_t ninst, uint64_t n, uint64_t* keys_out, void* vals_out, const Params& p,
                              uint32_t levels)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_OR_FAIL(c, hipStreamIsCapturing(c->stream, &cs));
    const bool capturing = cs != hipStreamCaptureStatusNone;
    ss_status s;
    DsPlan d;
    if ((s = ds_plan(c, n, ninst, p, &d)) != SS_OK) return s;
    size_t sz[kDsBufCount];
    ds_sizes(n, sizeof(V), d.b, levels, d.jtot, d.fcap, sz);
    DsSpace sp;
    if ((s = ds_space_ctx(c, sz, capturing, &sp)) != SS_OK) return s;
    if (!c->aux && capturing)
        return fail(c, SS_EINVAL, "the second stream must be created by an uncaptured call first");
    if ((s = ensure_aux(c)) != SS_OK) return s;
    return run_semisort_ds<MODE, V>(c, keys, vals, offs, ninst, n, keys_out, vals_out, p, levels, d, sp);
}

// The device-sized batch on the device's static scratch array (no allocation
// at all); SS_EINVAL when the call's worst case does not fit in it.
template <int MODE, typename V>
ss_status run_semisort_ds_static(ss_ctx* c, const uint64_t* keys, const void* vals, const uint64_t* offs,
                                 uint64_t ninst, uint64_t n, uint64_t* keys_out, void* vals_out, const Params& p,
                                 uint32_t levels)
{
    if (!c->scratch) return fail(c, SS_EHIP, "the static scratch array has no device address: " + c->scratch_err);
    if (!c->aux) return fail(c, SS_EHIP, "the context has no second stream");
    ss_status s;
    DsPlan d;
    if ((s = ds_plan(c, n, ninst, p, &d)) != SS_OK) return s;
    size_t sz[kDsBufCount];
    ds_sizes(n, sizeof(V), d.b, levels, d.jtot, d.fcap, sz);
    DsSpace sp;
    size_t need = 0;
    if (!ds_space_carve(c->scratch, kScratchBytes, sz, d.fcap, &sp, &need))
        return fail(c, SS_EINVAL, "the batch needs " + std::to_string(need) + " bytes of workspace, more than the " +
                                      std::to_string(kScratchBytes) + "-byte static scratch array holds");
    return run_semisort_ds<MODE, V>(c, keys, vals, offs, ninst, n, keys_out, vals_out, p, levels, d, sp);
}

// ---------------------------------------------------------------- collect-reduce

// Reduce-mode jobs of a level: base cases in LDS, sum jobs in the copy class.
template <int MODE, int ONES>
void launch_red_jobs_m(ss_ctx* c, const uint32_t* njobs, uint32_t cap, const uint64_t* sk, const uint64_t* sv,
                       uint64_t* rk, uint64_t* rv, uint8_t* rf, uint32_t op)
{
    const Job* jobs = (const Job*)c->jobs.p;
    if (njobs[0])
        hipLaunchKernelGGL((k_base_red<MODE, 1, ONES>), dim3(njobs[0]), dim3(64), 0, c->stream, jobs, sk, sv, rk, rv, rf,
                           op);
    if (njobs[1])
        hipLaunchKernelGGL((k_base_red<MODE, 2, ONES>), dim3(njobs[1]), dim3(128), 0, c->stream, jobs + cap, sk, sv, rk,
                           rv, rf, op);
    if (njobs[2])
        hipLaunchKernelGGL((k_base_red<MODE, 4, ONES>), dim3(njobs[2]), dim3(256), 0, c->stream, jobs + 2 * (size_t)cap,
                           sk, sv, rk, rv, rf, op);
    if (njobs[3])
        hipLaunchKernelGGL((k_base_red<MODE, 8, ONES>), dim3(njobs[3]), dim3(512), 0, c->stream, jobs + 3 * (size_t)cap,
                           sk, sv, rk, rv, rf, op);
    if (njobs[kCopyClass])
        hipLaunchKernelGGL((k_sum_job<ONES>), dim3(njobs[kCopyClass]), dim3(256), 0, c->stream,
                           jobs + (size_t)kCopyClass * cap, sk, sv, rk, rv, rf, op);
}

template <int RED>
void launch_red_jobs(ss_ctx* c, uint32_t mode, const uint32_t* njobs, uint32_t cap, const uint64_t* sk,
                     const uint64_t* sv, uint64_t* rk, uint64_t* rv, uint8_t* rf, uint64_t records, uint32_t op)
{
    ProfScope ps(c, SS_PROF_FINISH, records);
    if (mode == 1) launch_red_jobs_m<1, RED == 2>(c, njobs, cap, sk, sv, rk, rv, rf, op);
    else launch_red_jobs_m<0, RED == 2>(c, njobs, cap, sk, sv, rk, rv, rf, op);
}

template <int MODE, int RED>
void launch_red_level_m(ss_ctx* c, const LevelArgs& a, uint32_t tiles, uint32_t chunks, uint64_t records)
{
    {
        ProfScope ps(c, SS_PROF_SAMPLE, a.nsegs);
        hipLaunchKernelGGL((k_sample_heavy<MODE>), dim3(a.nsegs), dim3(1024), 0, c->stream, a);
    }
    {
        ProfScope ps(c, SS_PROF_COUNT, records);
        hipLaunchKernelGGL((k_count<MODE>), dim3(tiles), dim3(1024), 0, c->stream, a);
    }
    {
        ProfScope ps(c, SS_PROF_SCAN, tiles);
        hipLaunchKernelGGL(k_scan_chunks, dim3(chunks), dim3(256), 0, c->stream, a);
        hipLaunchKernelGGL(k_scan_buckets, dim3(a.nsegs * kBucketGroups), dim3(1024), 0, c->stream, a);
        hipLaunchKernelGGL(k_scan_offsets, dim3(a.nsegs), dim3(1024), 0, c->stream, a);
        hipLaunchKernelGGL(k_scan_fill, dim3(chunks), dim3(256), 0, c->stream, a);
    }
    {
        ProfScope ps(c, SS_PROF_DISTRIBUTE, records);
        hipLaunchKernelGGL((k_distribute<uint64_t, 16, 8, RED>), dim3(tiles), dim3(1024), 0, c->stream, a);
    }
    {
        ProfScope ps(c, SS_PROF_PLAN, a.nsegs);
        hipLaunchKernelGGL((k_heavy_results<MODE>), dim3(a.nsegs), dim3(256), 0, c->stream, a);
    }
}

// Collect-reduce (RED = 1, u64 values, wrapping sums) or histogram (RED = 2,
// no values) of n records.  Data moves between T and the caller's output
// arrays; results are written to T at positions flagged in rflag (positions
// of finished work are never touched again by later levels, which only work
// inside the ranges of unfinished buckets), then compacted into the output.
// Packs the results flagged in rf (position order) from (T_k, T_v) into the
// outputs and reads their number back (the buffers were sized by the caller:
// rf padded to whole flag blocks, bcnt and mdev as in run_reduce).
// m goes to d_m (device) when given, else to the context's own word; m_out
// (host), when given, receives it after a wait.  With m_out NULL the call
// does not wait.
ss_status compact_results(ss_ctx* c, uint64_t n, const uint64_t* T_k, const uint64_t* T_v, const uint8_t* rf,
                          uint64_t* out_keys, uint64_t* out_vals, uint64_t* m_out, uint64_t* d_m = nullptr)
{
    unsigned long long* mdst = d_m ? (unsigned long long*)d_m : (unsigned long long*)c->mdev.p;
    const uint64_t nblk = (n + kFlagBlock - 1) / kFlagBlock;
    const uint64_t nchunk = nblk * (kFlagBlock / kFlagChunk);
    {
        ProfScope ps(c, SS_PROF_COMPACT, n);
        uint32_t* ccnt = (uint32_t*)c->bcnt.p;  // per chunk, then per block
        uint32_t* btot = ccnt + nchunk;
        hipLaunchKernelGGL(k_flag_count, dim3((uint32_t)nblk), dim3(1024), 0, c->stream, rf, ccnt, btot);
        hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(1024), 0, c->stream, btot, (uint32_t)nblk, mdst);
        hipLaunchKernelGGL(k_flag_scatter, dim3((uint32_t)nblk), dim3(1024), 0, c->stream, rf, (const uint32_t*)ccnt,
                           (const uint32_t*)btot, n, T_k, T_v, out_keys, out_vals);
    }
    HIP_OR_FAIL(c, hipGetLastError());
    if (!m_out) return SS_OK;
    HIP_OR_FAIL(c, hipMemcpyAsync(c->info_host, c->info.p, sizeof(LevelInfo), hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(&c->info_host->records, mdst, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    if (c->info_host->status) return status_failure(c, c->info_host->status, "in collect-reduce");
    *m_out = c->info_host->records;
    return SS_OK;
}

// Collect-reduce (RED = 1, u64 values, the monoid `op`) or histogram (RED = 2,
// no values) of `ninst` independent instances packed back to back
// (instance i is [offs[i], offs[i+1]), host offsets).  Data moves between T
// and the caller's output arrays; results are written to T at positions
// flagged in rflag (positions of finished work are never touched again by
// later levels, which only work inside the ranges of unfinished buckets),
// then compacted into the outputs in position order, so every instance's
// pairs are contiguous and in the order the instance gives alone.
template <int RED>
ss_status run_reduce_multi(ss_ctx* c, const uint64_t* keys, const uint64_t* vals, const uint64_t* offs,
                           uint64_t ninst, uint64_t* out_keys, uint64_t* out_vals, uint64_t* m_out, const Params& p,
                           uint32_t op, uint64_t* d_m)
{
    c->call_tmaxd = 0;
    ss_status s;
    const uint64_t n = offs[ninst];
    const uint64_t nblk = (n + kFlagBlock - 1) / kFlagBlock;
    const uint64_t nchunk = nblk * (kFlagBlock / kFlagChunk);
    if ((s = ensure(c, c->t_keys, n * 8)) != SS_OK) return s;
    if ((s = ensure(c, c->t_vals, n * 8)) != SS_OK) return s;
    if ((s = ensure(c, c->rflag, nblk * kFlagBlock)) != SS_OK) return s;
    if ((s = ensure(c, c->bcnt, (nchunk + nblk) * 4)) != SS_OK) return s;
    if ((s = ensure(c, c->mdev, 8)) != SS_OK) return s;
    if ((s = ensure(c, c->info, sizeof(LevelInfo))) != SS_OK) return s;
    if ((s = ensure(c, c->sink, kSinkBytes)) != SS_OK) return s;
    // first level: instances of at least alpha records are subproblems, the
    // others base-case jobs (sum jobs for single records)
    std::vector<Seg> first;
    for (auto& v : c->host_jobs) v.clear();
    uint64_t jrec = 0;
    for (uint64_t i = 0; i < ninst; ++i) {
        const uint32_t st = (uint32_t)offs[i];
        const uint32_t len = (uint32_t)(offs[i + 1] - offs[i]);
        if (len >= p.alpha) {
            Seg sg{};
            sg.start = st;
            sg.len = len;
            sg.ibase = st;
            sg.nl_bits = (uint8_t)std::min(p.nl0, choose_nl(len, p.alpha, kLightBitsMax, 0));
            sg.shift = 0;
            first.push_back(sg);
        } else if (len >= 1) {
            c->host_jobs[len == 1 ? kCopyClass : base_class(len)].push_back(Job{st, len});
            jrec += len;
        }
    }
    uint32_t nj0[kJobClasses], nj0_max = 0, nj0_tot = 0;
    for (int k = 0; k < kJobClasses; ++k) {
        nj0[k] = (uint32_t)c->host_jobs[k].size();
        nj0_max = std::max(nj0_max, nj0[k]);
        nj0_tot += nj0[k];
    }
    if ((s = ensure_jobs(c, std::max<uint32_t>(nj0_max, 4096))) != SS_OK) return s;
    uint32_t seg_cap = std::max<uint32_t>((uint32_t)first.size(), 1024);
    if ((s = ensure(c, c->segs[0], (size_t)seg_cap * sizeof(Seg))) != SS_OK) return s;
    if ((s = ensure(c, c->segs[1], (size_t)seg_cap * sizeof(Seg))) != SS_OK) return s;
    seg_cap = (uint32_t)std::min(c->segs[0].cap, c->segs[1].cap) / sizeof(Seg);
    uint32_t nsegs = (uint32_t)first.size();
    uint32_t tiles = 0, chunks = 0, tile = p.tmin;
    uint64_t records = 0;
    for (const Seg& sg : first) records += sg.len;
    if (nsegs && (s = ensure(c, c->bids, n * 2)) != SS_OK) return s;
    uint64_t* T_k = (uint64_t*)c->t_keys.p;
    uint64_t* T_v = (uint64_t*)c->t_vals.p;
    uint8_t* rf = (uint8_t*)c->rflag.p;
    HIP_OR_FAIL(c, hipMemsetAsync(rf, 0, nblk * kFlagBlock, c->stream));
    if ((s = reset_counters(c)) != SS_OK) return s;
    const size_t stage = (size_t)nj0_tot * sizeof(Job) + (size_t)nsegs * sizeof(Seg);
    if ((s = stage_wait(c)) != SS_OK) return s;
    if (stage && (s = ensure_pinned(c, (void**)&c->job_stage, &c->job_stage_cap, stage)) != SS_OK) return s;
    if (nj0_tot) {
        size_t o = 0;
        for (int k = 0; k < kJobClasses; ++k) {
            if (!nj0[k]) continue;
            memcpy(c->job_stage + o, c->host_jobs[k].data(), nj0[k] * sizeof(Job));
            HIP_OR_FAIL(c, hipMemcpyAsync((Job*)c->jobs.p + (size_t)k * c->job_cap, c->job_stage + o,
                                          nj0[k] * sizeof(Job), hipMemcpyHostToDevice, c->stream));
            o += nj0[k];
        }
        launch_red_jobs<RED>(c, p.mode, nj0, c->job_cap, keys, vals, T_k, T_v, rf, jrec, op);
        HIP_OR_FAIL(c, hipGetLastError());
    }
    if (nsegs) {
        host_prefix(first, p, &tiles, &chunks, &tile);
        Seg* sst = (Seg*)(c->job_stage + nj0_tot);  // after the jobs in the same pinned staging
        memcpy(sst, first.data(), nsegs * sizeof(Seg));
        HIP_OR_FAIL(c, hipMemcpyAsync(c->segs[0].p, sst, nsegs * sizeof(Seg), hipMemcpyHostToDevice, c->stream));
    }
    if ((s = stage_mark(c)) != SS_OK) return s;
    if (nsegs) {
        int cur = 0;
        const uint64_t* loc_k = keys;
        const uint64_t* loc_v = vals;
        for (uint32_t level = 0; nsegs; ++level) {
            uint64_t* dst_k = loc_k == T_k ? out_keys : T_k;
            uint64_t* dst_v = loc_k == T_k ? out_vals : T_v;
            if ((s = ensure_level(c, nsegs, tiles, chunks)) != SS_OK) return s;
            if ((s = ensure(c, c->hsum, (size_t)nsegs * kHeavyMax * 8)) != SS_OK) return s;
            if ((s = reset_counters(c)) != SS_OK) return s;
            LevelArgs a = make_args(c, p, level, (Seg*)c->segs[cur].p, nsegs, tile, loc_k, loc_v, dst_k, dst_v, dst_k,
                                    dst_v);
            a.reduce = 1;
            a.hsum = (unsigned long long*)c->hsum.p;
            a.res_keys = T_k;
            a.res_vals = T_v;
            a.rflag = rf;
            a.rop = op;
            if (p.mode == 1) launch_red_level_m<1, RED>(c, a, tiles, chunks, records);
            else launch_red_level_m<0, RED>(c, a, tiles, chunks, records);
            HIP_OR_FAIL(c, hipGetLastError());
            LevelInfo li;
            if ((s = plan_level(c, p, level, nsegs, cur, &seg_cap, false, true, false, &li)) != SS_OK) return s;
            launch_red_jobs<RED>(c, p.mode, li.njobs, c->job_cap, dst_k, dst_v, T_k, T_v, rf, li.job_records, op);
            HIP_OR_FAIL(c, hipGetLastError());
            nsegs = li.nsegs;
            records = li.records;
            tiles = li.tiles;
            chunks = li.chunks;
            tile = li.tile;
            loc_k = dst_k;
            loc_v = dst_v;
            cur ^= 1;
        }
    }
    return compact_results(c, n, T_k, T_v, rf, out_keys, out_vals, m_out, d_m);
}

template <int RED>
ss_status run_reduce(ss_ctx* c, const uint64_t* keys, const uint64_t* vals, uint64_t n, uint64_t* out_keys,
                     uint64_t* out_vals, uint64_t* m_out, const Params& p, uint32_t op = 0, uint64_t* d_m = nullptr)
{
    const uint64_t offs[2] = {0, n};
    return run_reduce_multi<RED>(c, keys, vals, offs, 1, out_keys, out_vals, m_out, p, op, d_m);
}

ss_status check_reduce(ss_ctx* c, const uint64_t* keys, const uint64_t* vals, uint64_t n, const uint64_t* ok,
                       const uint64_t* ov, const uint64_t* m_out, const ss_params* params, Params* p)
{
    if (!c) return SS_EINVAL;
    if (!m_out) return fail(c, SS_EINVAL, "null m_out");
    if (n >= (1ull << 31)) return fail(c, SS_EINVAL, "n must be below 2^31");
    ss_status s = resolve_params(c, params, p);
    if (s != SS_OK) return s;
    if (n == 0) return SS_OK;
    if (!keys || !ok || !ov) return fail(c, SS_EINVAL, "null array pointer");
    const size_t b = n * 8;
    if (overlaps(ok, b, keys, b) || overlaps(ov, b, keys, b) || (vals && (overlaps(ok, b, vals, b) || overlaps(ov, b, vals, b))))
        return fail(c, SS_EINVAL, "outputs overlap inputs");
    if (overlaps(ok, b, ov, b)) return fail(c, SS_EINVAL, "out_keys overlaps the second output");
    return SS_OK;
}

ss_status check_common(ss_ctx* c, const void* keys, const void* vals, uint32_t vb, uint64_t n,
                       const void* ko, const void* vo, bool allow_inplace, uint32_t kb = 8)
{
    if (!c) return SS_EINVAL;
    if (vb != 4 && vb != 8) return fail(c, SS_EINVAL, "val_bytes must be 4 or 8");
    if (kb != 4 && kb != 8 && kb != 16) return fail(c, SS_EINVAL, "key_bytes must be 4, 8 or 16");
    if (n >= (1ull << 31)) return fail(c, SS_EINVAL, "n must be below 2^31");
    if (n == 0) return SS_OK;
    if (!keys || !vals || !ko || !vo) return fail(c, SS_EINVAL, "null array pointer");
    const bool inplace = ko == keys && vo == vals;
    if (inplace && !allow_inplace) return fail(c, SS_EINVAL, "in-place is not allowed here");
    if (!inplace) {
        if (ko == keys || vo == vals) return fail(c, SS_EINVAL, "in-place needs keys_out == keys and vals_out == vals");
        if (overlaps(ko, n * kb, keys, n * kb) || overlaps(ko, n * kb, vals, n * vb) ||
            overlaps(vo, n * vb, keys, n * kb) || overlaps(vo, n * vb, vals, n * vb))
            return fail(c, SS_EINVAL, "outputs overlap inputs");
    }
    if (overlaps(ko, n * kb, vo, n * vb)) return fail(c, SS_EINVAL, "keys_out overlaps vals_out");
    return SS_OK;
}

// Puts the m (key, result) pairs of a reduction into ascending key order: a
// semisort_< of the pairs in place (the keys are distinct, so its stable
// order is the sorted order), then a wait so the call keeps the reductions'
// convention of returning with its results ready.
ss_status order_results(ss_ctx* c, uint64_t* ok, uint64_t* ov, uint64_t m, const ss_params* params)
{
    if (m < 2) return SS_OK;
    Params p;
    ss_status s = resolve_params(c, params, &p);
    if (s != SS_OK) return s;
    p.mode = 2;
    default_tiles(c, params, &p, 32768u, 65536u);
    const uint64_t offs[2] = {0, m};
    if ((s = run_semisort<uint64_t>(c, ok, ov, offs, 1, ok, ov, p)) != SS_OK) return s;
    HIP_OR_FAIL(c, hipMemcpyAsync(c->info_host, c->info.p, sizeof(LevelInfo), hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    if (c->info_host->status) return status_failure(c, c->info_host->status, "in ordering the results");
    return SS_OK;
}

// Upper bound of the workspace that one call of `op` on n records can make a
// new context hold: every buffer the host-sized engine grows, at its largest
// size over all levels, with the headroom of ensure() (half again) on the
// buffers that grow level by level.  A level has at most n / alpha + 1
// subproblems (each holds at least alpha records), at most n / tile_min plus
// one per subproblem subarrays, and emits at most one job per bucket plus
// one per copy chunk.
size_t workspace_bound(int op, uint64_t n, uint32_t vb, const Params& p)
{
    if (n == 0) return 0;
    const bool reduce = op == SS_OP_HISTOGRAM || op == SS_OP_COLLECT_REDUCE;
    size_t b = 0;
    auto add = [&](uint64_t x) { b += (x + 255) & ~(uint64_t)255; };
    auto grow = [&](uint64_t x) { add(x + x / 2); };
    add(sizeof(LevelInfo));  // status word, held from ss_create
    add(kSinkBytes);         // sink
    add(n * 8);              // T: keys
    add(n * (reduce ? 8 : vb));  // T: values
    add(n * 2);              // bucket ids
    const uint64_t S = n / p.alpha + 1;
    const uint64_t tiles = n / p.tmin + S;
    const uint64_t chunks = tiles / kChunk + S;
    grow(tiles * kNbStride * 4);              // counting matrix
    grow(chunks * kNbStride * 4);             // chunk sums
    grow(S * kNbStride * 4);                  // bucket totals
    grow(S * (kNbStride + 1) * 4);            // bucket starts
    grow(S * kHeavyMax * 8);                  // heavy hashes
    grow(S * 2 * kHeavySlotsMax * 8);         // heavy tables: hashes
    grow(S * 2 * kHeavySlotsMax * 2);         // heavy tables: ids
    grow(S * kNbStride);                      // final-bucket flags
    grow(S * kNbStride * 8);                  // keys of one-key buckets
    grow(S * 4);                              // most sampled heavy buckets
    const uint64_t segs = std::max<uint64_t>(S, 1024) * sizeof(Seg);
    grow(segs);
    grow(segs);
    add(S * sizeof(Seg));                     // the list kept while both lists grow
    const uint64_t jobs = std::max<uint64_t>(4096, S * kNbStride + n / kCopyChunk + 1);
    grow(jobs * kJobClasses * sizeof(Job));
    if (reduce) {
        const uint64_t nblk = (n + kFlagBlock - 1) / kFlagBlock;
        add(nblk * kFlagBlock);                           // result flags
        add((nblk * (kFlagBlock / kFlagChunk) + nblk) * 4);  // flag counts
        add(8);                                           // m
        grow(S * kHeavyMax * 8);                          // heavy sums
    } else {
        const uint64_t f = std::max<uint64_t>(4096, S * kHeavyMax + n / kFillChunk + 1) * sizeof(FillJob);
        grow(f);  // key-fill lists of two levels
        grow(f);
    }
    return b;
}

}  // namespace

// ==================================================================== C-ABI

extern "C" {

ss_status ss_default_params(ss_params* p)
{
    if (!p) return SS_EINVAL;
    p->n_light_log2 = 10;
    p->base_case = kAlphaMax;
    p->sample_mult = 800;
    p->tile_min = 8192;
    p->tile_max = 0;  // by operation (equal_tiles)
    p->hash_mode = SS_HASH_MIX64;
    p->heavy_min = 3;
    p->temp_records = 0;
    p->seed = 0x5eed5eed2023ULL;
    return SS_OK;
}

ss_status ss_create(int device, void* hip_stream, size_t workspace_cap, ss_ctx** out)
{
    if (!out) return SS_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return SS_EHIP;
    ss_ctx* c = new (std::nothrow) ss_ctx();
    if (!c) return SS_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->ws_cap = workspace_cap;
    if (hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->ncu < 1)
        c->ncu = 1;
    if (hipHostMalloc((void**)&c->info_host, sizeof(LevelInfo), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return SS_EHIP;
    }
    if (ensure(c, c->info, sizeof(LevelInfo)) != SS_OK ||
        hipMemsetAsync(c->info.p, 0, sizeof(LevelInfo), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess || ensure_aux(c) != SS_OK ||
        hipEventCreateWithFlags(&c->stage_ev, hipEventDisableTiming) != hipSuccess) {
        (void)ss_destroy(c);
        return SS_EHIP;
    }
    // the static scratch array's address on this device (current above)
    const hipError_t se = scratch_address(device, &c->scratch);
    if (se != hipSuccess) {
        (void)hipGetLastError();
        c->scratch_err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(se);
    }
    *out = c;
    return SS_OK;
}

ss_status ss_destroy(ss_ctx* c)
{
    if (!c) return SS_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    DevBuf* bufs[] = {&c->t_keys, &c->t_vals, &c->segs[0], &c->segs[1], &c->jobs, &c->C, &c->P,
                      &c->tot, &c->bstart, &c->heavy_list, &c->tab_h, &c->tab_id, &c->info, &c->bids, &c->sink, &c->bfin,
                      &c->hsum, &c->rflag, &c->bcnt, &c->mdev, &c->bkey, &c->hrep, &c->top, &c->fills[0], &c->fills[1],
                      &c->wl_gk, &c->wl_gv, &c->wl_chunk, &c->wl_desc,
                      &c->ds_jobs, &c->ds_info, &c->ds_q,
                      &c->tr_keys, &c->tr_vals, &c->tr_sorted, &c->tr_min, &c->pos,
                      &c->pk_k, &c->pk_v, &c->po_k, &c->po_v, &c->pack_tab, &c->pack_rank};
    if (c->aux) (void)hipStreamSynchronize(c->aux);
    for (DevBuf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    for (auto& p : c->pending) {
        c->event_pool.push_back(p.a);
        c->event_pool.push_back(p.b);
    }
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->fill_done)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->fill_fork)
        if (e) (void)hipEventDestroy(e);
    if (c->plan_ev) (void)hipEventDestroy(c->plan_ev);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    if (c->info_host) (void)hipHostFree(c->info_host);
    if (c->seg_stage) (void)hipHostFree(c->seg_stage);
    if (c->job_stage) (void)hipHostFree(c->job_stage);
    if (c->pack_stage) (void)hipHostFree(c->pack_stage);
    if (c->stage_ev) (void)hipEventDestroy(c->stage_ev);
    delete c;
    return SS_OK;
}

ss_status ss_set_stream(ss_ctx* c, void* hip_stream)
{
    if (!c) return SS_EINVAL;
    c->stream = (hipStream_t)hip_stream;
    return SS_OK;
}

const char* ss_last_error(ss_ctx* c)
{
    return c ? c->err.c_str() : "null context";
}

ss_status ss_sync(ss_ctx* c)
{
    if (!c) return SS_EINVAL;
    HIP_OR_FAIL(c, hipMemcpyAsync(c->info_host, c->info.p, sizeof(LevelInfo), hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    if (c->info_host->status) return status_failure(c, c->info_host->status, "reported at ss_sync");
    return SS_OK;
}

ss_status ss_set_option(ss_ctx* c, int option, int64_t value)
{
    if (!c) return SS_EINVAL;
    switch (option) {
    case SS_OPT_DIST_VARIANT:
        if (value < 0 || value > 5) return fail(c, SS_EINVAL, "distribution variant must be 0..5");
        c->dist_variant = (int)value;
        return SS_OK;
    case SS_OPT_DEEP_SAMPLE_DIV:
        if (value < 1 || value > 64) return fail(c, SS_EINVAL, "deep sample divisor must be 1..64");
        c->deep_div = (uint32_t)value;
        return SS_OK;
    case SS_OPT_TILE0:
    case SS_OPT_TILE_DEEP: {
        const bool pw = value >= 8192 && value <= 65536 && (value & (value - 1)) == 0;
        if (value != 0 && !pw) return fail(c, SS_EINVAL, "tile limit must be 0 or a power of two in [8192, 65536]");
        (option == SS_OPT_TILE0 ? c->tile0 : c->tile_deep) = (uint32_t)value;
        return SS_OK;
    }
    case SS_OPT_FOLD_ROUND:
        if (value < 1 || value > 1024 || (value & (value - 1)) != 0)
            return fail(c, SS_EINVAL, "fold round must be a power of two in [1, 1024]");
        c->fold_round = (uint32_t)value;
        return SS_OK;
    case SS_OPT_NL_TARGET:
        if (value != 0 && (value < 10 || value > 100))
            return fail(c, SS_EINVAL, "light-bucket target must be 0 or 10..100 percent");
        c->nl_target = (uint32_t)value;
        return SS_OK;
    default:
        return fail(c, SS_EINVAL, "unknown option");
    }
}

ss_status ss_profile_enable(ss_ctx* c, int on)
{
    if (!c) return SS_EINVAL;
    ss_status s = resolve_profile(c);
    if (s != SS_OK) return s;
    for (int k = 0; k < SS_PROF_KINDS; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_launches[k] = 0;
        c->prof_units[k] = 0;
    }
    c->prof_on = on != 0;
    return SS_OK;
}

ss_status ss_profile_read(ss_ctx* c, int kind, double* total_ms, uint64_t* launches, uint64_t* units)
{
    if (!c || kind < 0 || kind >= SS_PROF_KINDS || !total_ms || !launches || !units) return SS_EINVAL;
    ss_status s = resolve_profile(c);
    if (s != SS_OK) return s;
    *total_ms = c->prof_ms[kind];
    *launches = c->prof_launches[kind];
    *units = c->prof_units[kind];
    return SS_OK;
}

ss_status ss_workspace_held(ss_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return SS_EINVAL;
    *bytes = c->ws_held;
    return SS_OK;
}

ss_status ss_workspace_bytes(int op, uint64_t n, uint32_t vb, const ss_params* params, size_t* bytes)
{
    if (!bytes) return SS_EINVAL;
    *bytes = 0;
    if (op < SS_OP_SEMISORT_EQUAL || op > SS_OP_COLLECT_REDUCE) return SS_EINVAL;
    const bool semisort = op == SS_OP_SEMISORT_EQUAL || op == SS_OP_SEMISORT_LESS;
    if (semisort && vb != 4 && vb != 8) return SS_EINVAL;
    if (n >= (1ull << 31)) return SS_EINVAL;
    Params p;
    if (resolve_params(nullptr, params, &p) != SS_OK) return SS_EINVAL;
    *bytes = workspace_bound(op, n, semisort ? vb : 8, p);
    return SS_OK;
}

ss_status ss_semisort_equal(ss_ctx* c, const uint64_t* keys, const void* vals, uint32_t vb, uint64_t n,
                            uint64_t* keys_out, void* vals_out, const ss_params* params)
{
    ss_status s = check_common(c, keys, vals, vb, n, keys_out, vals_out, true);
    if (s != SS_OK || n == 0) return s;
    Params p;
    if ((s = resolve_params(c, params, &p)) != SS_OK) return s;
    default_tiles(c, params, &p, 32768u, 16384u);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    const uint64_t offs[2] = {0, n};
    return vb == 8 ? run_semisort<uint64_t>(c, keys, vals, offs, 1, keys_out, vals_out, p)
                   : run_semisort<uint32_t>(c, keys, vals, offs, 1, keys_out, vals_out, p);
}

}  // extern "C"

// semisort_< of 128-bit keys (Section 2.1: groups in ascending key order,
// records of a key in input order): a stable semisort_= of the records puts
// every key's records in one run; the runs are numbered and sorted by key with
// two stable semisort_< passes over (word, run) pairs, low word first, so that
// the high word decides and the low word breaks its ties; a scatter then moves
// every record to its run's place in that order.  p holds the caller's hash
// mode for the semisort_=.
template <typename V>
ss_status run_less_wide(ss_ctx* c, const uint64_t* keys, const void* vals, uint64_t n, uint64_t* keys_out,
                        void* vals_out, const ss_params* params, const Params& p)
{
    ss_status s;
    if ((s = ensure(c, c->wl_gk, n * 16)) != SS_OK) return s;
    if ((s = ensure(c, c->wl_gv, n * sizeof(V))) != SS_OK) return s;
    Key128* gk = (Key128*)c->wl_gk.p;
    V* gv = (V*)c->wl_gv.p;
    {
        Params q = p;
        default_tiles(c, params, &q, 32768u, 16384u);
        const uint64_t offs[2] = {0, n};
        if ((s = run_semisort<V, Key128>(c, keys, vals, offs, 1, (uint64_t*)gk, gv, q)) != SS_OK) return s;
    }
    // runs of the grouped records
    const uint64_t nch = (n + kRunChunk - 1) / kRunChunk;
    // per chunk: its run count (scanned in place, then the total), and its
    // run-start bitmap of kRunWords words
    if ((s = ensure(c, c->wl_chunk, (nch + 2 + nch * kRunWords) * 4)) != SS_OK) return s;
    uint32_t* chunk = (uint32_t*)c->wl_chunk.p;
    uint32_t* dtotal = chunk + nch;
    uint32_t* bits = chunk + nch + 2;
    hipLaunchKernelGGL(k_runs_count, dim3((uint32_t)nch), dim3(256), 0, c->stream, (const Key128*)gk, n, chunk, bits);
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, c->stream, chunk, (uint32_t)nch, dtotal);
    HIP_OR_FAIL(c, hipGetLastError());
    uint32_t m = 0;
    HIP_OR_FAIL(c, hipMemcpyAsync(c->info_host, dtotal, 4, hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    memcpy(&m, c->info_host, 4);
    if (m == 0 || m > n) return fail(c, SS_EINVAL, "run count out of range");
    // per run: start, words, and the arrays of the two sorts
    const uint64_t mch = (m + kRunChunk - 1) / kRunChunk;
    auto al = [](uint64_t b) { return (b + 255) & ~(uint64_t)255; };
    const uint64_t o_gstart = 0, o_glo = o_gstart + al(m * 4ull), o_ghi = o_glo + al(m * 8ull),
                   o_idx = o_ghi + al(m * 8ull), o_slo = o_idx + al(m * 4ull), o_sidx = o_slo + al(m * 8ull),
                   o_len = o_sidx + al(m * 4ull), o_dest = o_len + al(m * 4ull), o_csum = o_dest + al(m * 4ull),
                   o_end = o_csum + al((mch + 2) * 4);
    if ((s = ensure(c, c->wl_desc, o_end)) != SS_OK) return s;
    char* d = (char*)c->wl_desc.p;
    uint32_t* gstart = (uint32_t*)(d + o_gstart);
    uint64_t* glo = (uint64_t*)(d + o_glo);
    uint64_t* ghi = (uint64_t*)(d + o_ghi);
    uint32_t* idx = (uint32_t*)(d + o_idx);
    uint64_t* slo = (uint64_t*)(d + o_slo);
    uint32_t* sidx = (uint32_t*)(d + o_sidx);
    uint32_t* len = (uint32_t*)(d + o_len);
    uint32_t* dest = (uint32_t*)(d + o_dest);
    uint32_t* csum = (uint32_t*)(d + o_csum);
    const uint32_t gm = (uint32_t)std::min<uint64_t>((m + 255) / 256, 65536);
    hipLaunchKernelGGL(k_runs_emit, dim3((uint32_t)nch), dim3(256), 0, c->stream, (const Key128*)gk, n,
                       (const uint32_t*)chunk, (const uint32_t*)bits, gstart, glo, ghi);
    hipLaunchKernelGGL(k_iota_u32, dim3(gm), dim3(256), 0, c->stream, idx, m);
    HIP_OR_FAIL(c, hipGetLastError());
    // the runs in key order: by low word, then (stably) by high word
    Params q = p;
    q.mode = 2;
    default_tiles(c, params, &q, 32768u, 65536u);
    const uint64_t mo[2] = {0, m};
    if ((s = run_semisort<uint32_t>(c, glo, idx, mo, 1, slo, sidx, q)) != SS_OK) return s;
    hipLaunchKernelGGL(k_gather_u64_u32, dim3(gm), dim3(256), 0, c->stream, (const uint64_t*)ghi,
                       (const uint32_t*)sidx, m, glo);
    HIP_OR_FAIL(c, hipGetLastError());
    uint32_t* order = idx;  // the second sort's values land where the run numbers were
    if ((s = run_semisort<uint32_t>(c, glo, sidx, mo, 1, slo, order, q)) != SS_OK) return s;
    // destinations of the runs, then every record to its place
    hipLaunchKernelGGL(k_runs_lens, dim3(gm), dim3(256), 0, c->stream, (const uint32_t*)order,
                       (const uint32_t*)gstart, m, n, len);
    hipLaunchKernelGGL(k_sum_chunks_u32, dim3((uint32_t)mch), dim3(256), 0, c->stream, (const uint32_t*)len, m, csum);
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, c->stream, csum, (uint32_t)mch, csum + mch);
    hipLaunchKernelGGL(k_runs_dest, dim3((uint32_t)mch), dim3(256), 0, c->stream, (const uint32_t*)len,
                       (const uint32_t*)order, m, (const uint32_t*)csum, dest);
    hipLaunchKernelGGL((k_runs_scatter<V>), dim3((uint32_t)nch), dim3(256), 0, c->stream, (const Key128*)gk,
                       (const V*)gv, n, (const uint32_t*)chunk, (const uint32_t*)bits, (const uint32_t*)gstart,
                       (const uint32_t*)dest, (Key128*)keys_out, (V*)vals_out);
    HIP_OR_FAIL(c, hipGetLastError());
    return SS_OK;
}

extern "C" {

// semisort_= / semisort_< with keys of key_bytes bytes: 4 or 8, or 16 for
// semisort_= (the two words of a 128-bit key, low word first, 16-byte aligned).
static ss_status semisort_keys(ss_ctx* c, bool less, const void* keys, uint32_t kb, const void* vals, uint32_t vb,
                               uint64_t n, void* keys_out, void* vals_out, const ss_params* params)
{
    if (c && kb == 16 && (((uintptr_t)keys | (uintptr_t)keys_out) & 15u))
        return fail(c, SS_EINVAL, "16-byte keys must be 16-byte aligned");
    ss_status s = check_common(c, keys, vals, vb, n, keys_out, vals_out, true, kb);
    if (s != SS_OK || n == 0) return s;
    Params p;
    if ((s = resolve_params(c, params, &p)) != SS_OK) return s;
    if (less && kb == 16) {
        if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
        return vb == 8 ? run_less_wide<uint64_t>(c, (const uint64_t*)keys, vals, n, (uint64_t*)keys_out, vals_out,
                                                 params, p)
                       : run_less_wide<uint32_t>(c, (const uint64_t*)keys, vals, n, (uint64_t*)keys_out, vals_out,
                                                 params, p);
    }
    if (less) {
        p.mode = 2;
        default_tiles(c, params, &p, 32768u, 65536u);
    } else {
        default_tiles(c, params, &p, 32768u, 16384u);
    }
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    const uint64_t offs[2] = {0, n};
    const uint64_t* k = (const uint64_t*)keys;
    uint64_t* ko = (uint64_t*)keys_out;
    if (kb == 4)
        return vb == 8 ? run_semisort<uint64_t, uint32_t>(c, k, vals, offs, 1, ko, vals_out, p)
                       : run_semisort<uint32_t, uint32_t>(c, k, vals, offs, 1, ko, vals_out, p);
    if (kb == 16)
        return vb == 8 ? run_semisort<uint64_t, Key128>(c, k, vals, offs, 1, ko, vals_out, p)
                       : run_semisort<uint32_t, Key128>(c, k, vals, offs, 1, ko, vals_out, p);
    return vb == 8 ? run_semisort<uint64_t>(c, k, vals, offs, 1, ko, vals_out, p)
                   : run_semisort<uint32_t>(c, k, vals, offs, 1, ko, vals_out, p);
}

ss_status ss_semisort_equal_keys(ss_ctx* c, const void* keys, uint32_t key_bytes, const void* vals, uint32_t vb,
                                 uint64_t n, void* keys_out, void* vals_out, const ss_params* params)
{
    return semisort_keys(c, false, keys, key_bytes, vals, vb, n, keys_out, vals_out, params);
}

ss_status ss_semisort_less_keys(ss_ctx* c, const void* keys, uint32_t key_bytes, const void* vals, uint32_t vb,
                                uint64_t n, void* keys_out, void* vals_out, const ss_params* params)
{
    return semisort_keys(c, true, keys, key_bytes, vals, vb, n, keys_out, vals_out, params);
}

ss_status ss_semisort_equal_batch(ss_ctx* c, const uint64_t* keys, const void* vals, uint32_t vb,
                                  const uint64_t* offs, uint64_t nseg, uint64_t* keys_out, void* vals_out,
                                  const ss_params* params)
{
    if (!c) return SS_EINVAL;
    if (!offs) return fail(c, SS_EINVAL, "null seg_offsets");
    if (nseg == 0) return SS_OK;
    if (offs[0] != 0) return fail(c, SS_EINVAL, "seg_offsets[0] must be 0");
    for (uint64_t i = 0; i < nseg; ++i)
        if (offs[i + 1] < offs[i]) return fail(c, SS_EINVAL, "seg_offsets must be non-decreasing");
    const uint64_t n = offs[nseg];
    ss_status s = check_common(c, keys, vals, vb, n, keys_out, vals_out, true);
    if (s != SS_OK || n == 0) return s;
    Params p;
    if ((s = resolve_params(c, params, &p)) != SS_OK) return s;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    return vb == 8 ? run_semisort<uint64_t>(c, keys, vals, offs, nseg, keys_out, vals_out, p)
                   : run_semisort<uint32_t>(c, keys, vals, offs, nseg, keys_out, vals_out, p);
}

ss_status ss_semisort_equal_batch_capturable(ss_ctx* c, const uint64_t* keys, const void* vals, uint32_t vb,
                                             const uint64_t* seg_offsets, uint64_t nseg, uint64_t n,
                                             uint64_t* keys_out, void* vals_out, uint32_t max_levels,
                                             const ss_params* params)
{
    if (!c) return SS_EINVAL;
    if (nseg == 0) return SS_OK;
    if (!seg_offsets) return fail(c, SS_EINVAL, "null seg_offsets");
    if (nseg >= (1ull << 31)) return fail(c, SS_EINVAL, "too many instances");
    if (max_levels < 1 || max_levels > 64) return fail(c, SS_EINVAL, "max_levels must be in 1..64");
    ss_status s = check_common(c, keys, vals, vb, n, keys_out, vals_out, true);
    if (s != SS_OK || n == 0) return s;
    Params p;
    if ((s = resolve_params(c, params, &p)) != SS_OK) return s;
    default_tiles(c, params, &p, 32768u, 16384u);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    if (p.mode == 1)
        return vb == 8 ? run_semisort_ds_ctx<1, uint64_t>(c, keys, vals, seg_offsets, nseg, n, keys_out, vals_out, p, max_levels)
                       : run_semisort_ds_ctx<1, uint32_t>(c, keys, vals, seg_offsets, nseg, n, keys_out, vals_out, p, max_levels);
    return vb == 8 ? run_semisort_ds_ctx<0, uint64_t>(c, keys, vals, seg_offsets, nseg, n, keys_out, vals_out, p, max_levels)
                   : run_semisort_ds_ctx<0, uint32_t>(c, keys, vals, seg_offsets, nseg, n, keys_out, vals_out, p, max_levels);
}

ss_status ss_semisort_equal_batch_noalloc(ss_ctx* c, const uint64_t* keys, const void* vals, uint32_t vb,
                                          const uint64_t* seg_offsets, uint64_t nseg, uint64_t n,
                                          uint64_t* keys_out, void* vals_out, uint32_t max_levels,
                                          const ss_params* params)
{
    if (!c) return SS_EINVAL;
    if (nseg == 0) return SS_OK;
    if (!seg_offsets) return fail(c, SS_EINVAL, "null seg_offsets");
    if (nseg >= (1ull << 31)) return fail(c, SS_EINVAL, "too many instances");
    if (max_levels < 1 || max_levels > 64) return fail(c, SS_EINVAL, "max_levels must be in 1..64");
    ss_status s = check_common(c, keys, vals, vb, n, keys_out, vals_out, true);
    if (s != SS_OK || n == 0) return s;
    Params p;
    if ((s = resolve_params(c, params, &p)) != SS_OK) return s;
    default_tiles(c, params, &p, 32768u, 16384u);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    if (p.mode == 1)
        return vb == 8 ? run_semisort_ds_static<1, uint64_t>(c, keys, vals, seg_offsets, nseg, n, keys_out, vals_out, p, max_levels)
                       : run_semisort_ds_static<1, uint32_t>(c, keys, vals, seg_offsets, nseg, n, keys_out, vals_out, p, max_levels);
    return vb == 8 ? run_semisort_ds_static<0, uint64_t>(c, keys, vals, seg_offsets, nseg, n, keys_out, vals_out, p, max_levels)
                   : run_semisort_ds_static<0, uint32_t>(c, keys, vals, seg_offsets, nseg, n, keys_out, vals_out, p, max_levels);
}

ss_status ss_autotune_equal_batch(ss_ctx* c, const uint64_t* keys, const void* vals, uint32_t vb,
                                  const uint64_t* offs, uint64_t nseg, uint64_t* keys_out, void* vals_out,
                                  uint32_t reps, ss_params* best, double* best_ms)
{
    if (!c) return SS_EINVAL;
    if (!offs || !best || !best_ms) return fail(c, SS_EINVAL, "null argument");
    if (nseg == 0) return fail(c, SS_EINVAL, "nothing to tune on");
    if (offs[0] != 0) return fail(c, SS_EINVAL, "seg_offsets[0] must be 0");
    for (uint64_t i = 0; i < nseg; ++i)
        if (offs[i + 1] < offs[i]) return fail(c, SS_EINVAL, "seg_offsets must be non-decreasing");
    const uint64_t n = offs[nseg];
    ss_status s = check_common(c, keys, vals, vb, n, keys_out, vals_out, false);
    if (s != SS_OK) return s;
    if (n == 0) return fail(c, SS_EINVAL, "nothing to tune on");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    if (reps < 1) reps = 1;
    // candidate grid around the defaults: sample multiplier, heavy threshold,
    // light-bucket cap, base-case size and largest subarray
    std::vector<ss_params> cand;
    const uint32_t cs[] = {500, 800};
    const uint32_t taus[] = {0, 3};
    const uint32_t nls[] = {8, 10};
    const uint32_t alphas[] = {2048, 4096};
    const uint32_t tmaxs[] = {32768, 65536};
    for (uint32_t cc : cs)
        for (uint32_t tau : taus)
            for (uint32_t nl : nls)
                for (uint32_t al : alphas)
                    for (uint32_t tm : tmaxs) {
                        ss_params q;
                        ss_default_params(&q);
                        q.sample_mult = cc;
                        q.heavy_min = tau;
                        q.n_light_log2 = nl;
                        q.base_case = al;
                        q.tile_max = tm;
                        cand.push_back(q);
                    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OR_FAIL(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, SS_EHIP, "hipEventCreate");
    }
    auto run = [&](const ss_params& q, float* ms) -> ss_status {
        Params p;
        ss_status r = resolve_params(c, &q, &p);
        if (r != SS_OK) return r;
        if (hipEventRecord(e0, c->stream) != hipSuccess) return fail(c, SS_EHIP, "hipEventRecord");
        for (uint32_t k = 0; k < reps; ++k) {
            r = vb == 8 ? run_semisort<uint64_t>(c, keys, vals, offs, nseg, keys_out, vals_out, p)
                        : run_semisort<uint32_t>(c, keys, vals, offs, nseg, keys_out, vals_out, p);
            if (r != SS_OK) return r;
        }
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            return fail(c, SS_EHIP, "timing");
        *ms /= (float)reps;
        return SS_OK;
    };
    float ms = 0.f, best_t = 0.f;
    size_t bi = 0;
    s = run(cand[0], &ms);  // warm-up: grows the workspace once
    for (size_t i = 0; s == SS_OK && i < cand.size(); ++i) {
        s = run(cand[i], &ms);
        if (s == SS_OK && (i == 0 || ms < best_t)) {
            best_t = ms;
            bi = i;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != SS_OK) return s;
    if ((s = ss_sync(c)) != SS_OK) return s;
    *best = cand[bi];
    *best_ms = best_t;
    return SS_OK;
}

// Class of a batch for the autotuned parameters: the operation, key and value
// widths, and the binary orders of the total size and of the mean instance size.
static uint64_t batch_class(int op, uint32_t kb, uint32_t vb, uint64_t n, uint64_t nseg)
{
    auto lg = [](uint64_t x) -> uint64_t { return x ? 63 - (uint64_t)__builtin_clzll(x) : 0; };
    return ((uint64_t)op << 40) | ((uint64_t)kb << 32) | ((uint64_t)vb << 24) | (lg(n) << 8) |
           lg(nseg ? n / nseg : 0);
}

ss_status ss_semisort_equal_batch_tuned(ss_ctx* c, const uint64_t* keys, const void* vals, uint32_t vb,
                                        const uint64_t* offs, uint64_t nseg, uint64_t* keys_out, void* vals_out,
                                        ss_params* used, int* tuned_now)
{
    if (!c) return SS_EINVAL;
    if (!offs) return fail(c, SS_EINVAL, "null seg_offsets");
    if (nseg == 0) return fail(c, SS_EINVAL, "empty batch");
    const uint64_t cls = batch_class(SS_OP_SEMISORT_EQUAL, 8, vb, offs[nseg], nseg);
    auto it = c->tuned.find(cls);
    ss_status s;
    if (it == c->tuned.end()) {
        ss_params best;
        double ms = 0;
        if ((s = ss_autotune_equal_batch(c, keys, vals, vb, offs, nseg, keys_out, vals_out, 1, &best, &ms)) != SS_OK)
            return s;
        c->tuned[cls] = best;
        if (used) *used = best;
        if (tuned_now) *tuned_now = 1;
        return SS_OK;
    }
    if (used) *used = it->second;
    if (tuned_now) *tuned_now = 0;
    return ss_semisort_equal_batch(c, keys, vals, vb, offs, nseg, keys_out, vals_out, &it->second);
}

ss_status ss_autotune_cache(ss_ctx* c, int clear, uint64_t* entries)
{
    if (!c) return SS_EINVAL;
    if (clear) c->tuned.clear();
    if (entries) *entries = c->tuned.size();
    return SS_OK;
}

ss_status ss_semisort_less(ss_ctx* c, const uint64_t* keys, const void* vals, uint32_t vb, uint64_t n,
                           uint64_t* keys_out, void* vals_out, const ss_params* params)
{
    ss_status s = check_common(c, keys, vals, vb, n, keys_out, vals_out, true);
    if (s != SS_OK || n == 0) return s;
    Params p;
    if ((s = resolve_params(c, params, &p)) != SS_OK) return s;
    p.mode = 2;
    default_tiles(c, params, &p, 32768u, 65536u);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    const uint64_t offs[2] = {0, n};
    return vb == 8 ? run_semisort<uint64_t>(c, keys, vals, offs, 1, keys_out, vals_out, p)
                   : run_semisort<uint32_t>(c, keys, vals, offs, 1, keys_out, vals_out, p);
}

ss_status ss_semisort_less_batch(ss_ctx* c, const uint64_t* keys, const void* vals, uint32_t vb,
                                 const uint64_t* offs, uint64_t nseg, uint64_t* keys_out, void* vals_out,
                                 const ss_params* params)
{
    if (!c) return SS_EINVAL;
    if (!offs) return fail(c, SS_EINVAL, "null seg_offsets");
    if (nseg == 0) return SS_OK;
    if (offs[0] != 0) return fail(c, SS_EINVAL, "seg_offsets[0] must be 0");
    for (uint64_t i = 0; i < nseg; ++i)
        if (offs[i + 1] < offs[i]) return fail(c, SS_EINVAL, "seg_offsets must be non-decreasing");
    const uint64_t n = offs[nseg];
    ss_status s = check_common(c, keys, vals, vb, n, keys_out, vals_out, true);
    if (s != SS_OK || n == 0) return s;
    Params p;
    if ((s = resolve_params(c, params, &p)) != SS_OK) return s;
    p.mode = 2;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    return vb == 8 ? run_semisort<uint64_t>(c, keys, vals, offs, nseg, keys_out, vals_out, p)
                   : run_semisort<uint32_t>(c, keys, vals, offs, nseg, keys_out, vals_out, p);
}

ss_status ss_partition_equal(ss_ctx* c, const uint64_t* keys, const void* vals, uint32_t vb, uint64_t n,
                             uint64_t* keys_out, void* vals_out, uint64_t* offsets_out,
                             uint64_t* heavy_out, uint32_t* n_heavy_out, const ss_params* params)
{
    ss_status s = check_common(c, keys, vals, vb, n, keys_out, vals_out, false);
    if (s != SS_OK) return s;
    if (!offsets_out || !heavy_out || !n_heavy_out) return fail(c, SS_EINVAL, "null output pointer");
    if (n == 0) return fail(c, SS_EINVAL, "partition needs n >= 1");
    Params p;
    if ((s = resolve_params(c, params, &p)) != SS_OK) return s;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    std::vector<Seg> segs(1);
    segs[0] = Seg{};
    segs[0].start = 0;
    segs[0].len = (uint32_t)n;
    segs[0].ibase = 0;
    segs[0].nl_bits = (uint8_t)p.nl0;
    segs[0].shift = 0;
    uint32_t tiles, chunks, tile;
    host_prefix(segs, p, &tiles, &chunks, &tile);
    if ((s = ensure(c, c->info, sizeof(LevelInfo))) != SS_OK) return s;
    if ((s = ensure(c, c->segs[0], sizeof(Seg))) != SS_OK) return s;
    if ((s = ensure_level(c, 1, tiles, chunks)) != SS_OK) return s;
    if ((s = ensure_pinned(c, (void**)&c->seg_stage, &c->seg_stage_cap, sizeof(Seg))) != SS_OK) return s;
    memcpy(c->seg_stage, segs.data(), sizeof(Seg));
    HIP_OR_FAIL(c, hipMemcpyAsync(c->segs[0].p, c->seg_stage, sizeof(Seg), hipMemcpyHostToDevice, c->stream));
    if ((s = reset_counters(c)) != SS_OK) return s;
    if ((s = ensure(c, c->bids, n * 2)) != SS_OK) return s;
    if ((s = ensure(c, c->sink, kSinkBytes)) != SS_OK) return s;
    LevelArgs a = make_args(c, p, 0, (Seg*)c->segs[0].p, 1, tile, keys, vals, keys_out, vals_out, keys_out, vals_out);
    a.adaptive_nl = 0;  // the inspected level uses exactly n_light_log2 bits
    if (vb == 8) launch_level_v<uint64_t>(c, p.mode, a, tiles, chunks, n);
    else launch_level_v<uint32_t>(c, p.mode, a, tiles, chunks, n);
    hipLaunchKernelGGL(k_export_partition, dim3(1), dim3(1024), 0, c->stream, (const uint32_t*)c->bstart.p,
                       (const Seg*)c->segs[0].p, (const uint64_t*)c->heavy_list.p, offsets_out, heavy_out);
    HIP_OR_FAIL(c, hipGetLastError());
    Seg back;
    HIP_OR_FAIL(c, hipMemcpyAsync(c->seg_stage, c->segs[0].p, sizeof(Seg), hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(c->info_host, c->info.p, sizeof(LevelInfo), hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    memcpy(&back, c->seg_stage, sizeof(Seg));
    if (c->info_host->status) return status_failure(c, c->info_host->status, "in the partition");
    *n_heavy_out = back.nheavy;
    return SS_OK;
}

ss_status ss_collect_reduce(ss_ctx* c, const uint64_t* keys, const uint64_t* vals, uint64_t n, uint64_t* out_keys,
                            uint64_t* out_sums, uint64_t* m_out, const ss_params* params)
{
    Params p;
    ss_status s = check_reduce(c, keys, vals, n, out_keys, out_sums, m_out, params, &p);
    if (s != SS_OK) return s;
    *m_out = 0;
    if (n == 0) return SS_OK;
    if (!vals) return fail(c, SS_EINVAL, "null vals");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    return run_reduce<1>(c, keys, vals, n, out_keys, out_sums, m_out, p);
}

ss_status ss_histogram(ss_ctx* c, const uint64_t* keys, uint64_t n, uint64_t* out_keys, uint64_t* out_counts,
                       uint64_t* m_out, const ss_params* params)
{
    Params p;
    ss_status s = check_reduce(c, keys, nullptr, n, out_keys, out_counts, m_out, params, &p);
    if (s != SS_OK) return s;
    *m_out = 0;
    if (n == 0) return SS_OK;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    return run_reduce<2>(c, keys, nullptr, n, out_keys, out_counts, m_out, p);
}

ss_status ss_transpose_csr(ss_ctx* c, uint64_t nv, uint64_t ne, const uint64_t* offs, const uint32_t* cols,
                           uint64_t* out_offs, uint32_t* out_cols, const ss_params* params)
{
    if (!c) return SS_EINVAL;
    if (nv >= (1ull << 32)) return fail(c, SS_EINVAL, "vertex ids must fit in 32 bits");
    if (ne >= (1ull << 31)) return fail(c, SS_EINVAL, "ne must be below 2^31");
    if (!offs || !out_offs || (ne && (!cols || !out_cols))) return fail(c, SS_EINVAL, "null array pointer");
    if (ne && nv == 0) return fail(c, SS_EINVAL, "edges without vertices");
    if (ne && (overlaps(out_cols, ne * 4, cols, ne * 4) || overlaps(out_offs, (nv + 1) * 8, offs, (nv + 1) * 8) ||
               overlaps(out_offs, (nv + 1) * 8, out_cols, ne * 4)))
        return fail(c, SS_EINVAL, "outputs overlap inputs or each other");
    Params p;
    ss_status s = resolve_params(c, params, &p);
    if (s != SS_OK) return s;
    p.mode = 2;
    default_tiles(c, params, &p, 32768u, 65536u);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    if ((s = ensure(c, c->info, sizeof(LevelInfo))) != SS_OK) return s;
    if ((s = reset_counters(c)) != SS_OK) return s;
    // the CSR's ends, read once: offs[0] = 0 and offs[nv] = ne
    uint64_t ends[2] = {1, 0};
    HIP_OR_FAIL(c, hipMemcpyAsync(&ends[0], offs, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(&ends[1], offs + nv, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    if (ends[0] != 0 || ends[1] != ne) return fail(c, SS_EINVAL, "offsets must start at 0 and end at ne");
    uint64_t* out = out_offs;
    const uint64_t n = nv + 1;
    const uint64_t nb = (n + kMinChunk - 1) / kMinChunk;
    if ((s = ensure(c, c->tr_min, nb * 8)) != SS_OK) return s;
    LevelInfo* info = (LevelInfo*)c->info.p;
    uint64_t* sk = nullptr;
    if (ne) {
        if ((s = ensure(c, c->tr_keys, ne * 8)) != SS_OK) return s;
        if ((s = ensure(c, c->tr_vals, ne * 4)) != SS_OK) return s;
        if ((s = ensure(c, c->tr_sorted, ne * 8)) != SS_OK) return s;
        uint64_t* tk = (uint64_t*)c->tr_keys.p;
        uint32_t* tv = (uint32_t*)c->tr_vals.p;
        sk = (uint64_t*)c->tr_sorted.p;
        hipLaunchKernelGGL(k_csr_check, dim3((uint32_t)std::min<uint64_t>((nv + 255) / 256, 65536)), dim3(256), 0,
                           c->stream, offs, (uint32_t)nv, info);
        hipLaunchKernelGGL(k_csr_expand, dim3((uint32_t)((ne + kExpandEdges - 1) / kExpandEdges)), dim3(256), 0,
                           c->stream, offs, cols, (uint32_t)nv, ne, tk, tv, info);
        HIP_OR_FAIL(c, hipGetLastError());
        // the transpose proper: a stable semisort_< by the other endpoint
        const uint64_t so[2] = {0, ne};
        if ((s = run_semisort<uint32_t>(c, tk, tv, so, 1, sk, out_cols, p)) != SS_OK) return s;
    }
    hipLaunchKernelGGL(k_csr_init, dim3((uint32_t)std::min<uint64_t>((n + 255) / 256, 65536)), dim3(256), 0,
                       c->stream, out, (uint32_t)nv, ne);
    if (ne)
        hipLaunchKernelGGL(k_csr_starts, dim3((uint32_t)std::min<uint64_t>((ne + 255) / 256, 65536)), dim3(256), 0,
                           c->stream, (const uint64_t*)sk, ne, (uint32_t)nv, out, info);
    hipLaunchKernelGGL(k_min_chunks, dim3((uint32_t)nb), dim3(256), 0, c->stream, (const uint64_t*)out, n,
                       (uint64_t*)c->tr_min.p);
    hipLaunchKernelGGL(k_min_carry, dim3(1), dim3(1024), 0, c->stream, (uint64_t*)c->tr_min.p, (uint32_t)nb);
    hipLaunchKernelGGL(k_min_fill, dim3((uint32_t)nb), dim3(256), 0, c->stream, out, n,
                       (const uint64_t*)c->tr_min.p);
    HIP_OR_FAIL(c, hipGetLastError());
    return ss_sync(c);
}

// collect-reduce with a monoid after the argument checks (n >= 1): m goes to
// *m_out (host, after a wait) when m_out is given, and to d_m (device) when
// d_m is given; with m_out NULL and ordered = 0 nothing waits for the result.
static ss_status reduce_call(ss_ctx* c, const uint64_t* keys, const uint64_t* vals, uint64_t n, int op, int ordered,
                      uint64_t* out_keys, uint64_t* out_vals, uint64_t* m_out, uint64_t* d_m, const ss_params* params,
                      const Params& p)
{
    ss_status s;
    uint64_t m_host = 0;
    if (ordered && !m_out) m_out = &m_host;  // ordering the pairs needs m on the host
    if (op == SS_MONOID_AFFINE) {
        // in input order: a stable semisort_= makes every key's records
        // contiguous and ordered, then a segmented scan folds each group
        Params q = p;
        default_tiles(c, params, &q, 32768u, 16384u);
        if ((s = ensure(c, c->tr_keys, n * 8)) != SS_OK) return s;
        if ((s = ensure(c, c->tr_sorted, n * 8)) != SS_OK) return s;
        uint64_t* sk = (uint64_t*)c->tr_keys.p;
        uint64_t* sv = (uint64_t*)c->tr_sorted.p;
        const uint64_t so[2] = {0, n};
        if ((s = run_semisort<uint64_t>(c, keys, vals, so, 1, sk, sv, q)) != SS_OK) return s;
        const uint64_t nblk = (n + kFlagBlock - 1) / kFlagBlock;
        const uint64_t nch = (n + kFoldChunk - 1) / kFoldChunk;
        if ((s = ensure(c, c->t_keys, n * 8)) != SS_OK) return s;
        if ((s = ensure(c, c->t_vals, n * 8)) != SS_OK) return s;
        if ((s = ensure(c, c->rflag, nblk * kFlagBlock)) != SS_OK) return s;
        if ((s = ensure(c, c->bcnt, (nblk * (kFlagBlock / kFlagChunk) + nblk) * 4)) != SS_OK) return s;
        if ((s = ensure(c, c->mdev, 8)) != SS_OK) return s;
        const uint64_t ncb = (nch + 255) / 256;  // blocks of the first carry level (<= 2048 for n < 2^31)
        if ((s = ensure(c, c->pos, (nch + ncb) * 12)) != SS_OK) return s;
        uint64_t* aggv = (uint64_t*)c->pos.p;
        uint64_t* totv = aggv + nch;
        uint32_t* aggf = (uint32_t*)(totv + ncb);
        uint32_t* totf = aggf + nch;
        uint8_t* rf = (uint8_t*)c->rflag.p;
        HIP_OR_FAIL(c, hipMemsetAsync(rf, 0, nblk * kFlagBlock, c->stream));
        hipLaunchKernelGGL(k_sfold_aggr, dim3((uint32_t)nch), dim3(256), 0, c->stream, (const uint64_t*)sk,
                           (const uint64_t*)sv, n, aggv, aggf);
        hipLaunchKernelGGL(k_sfold_carry_blocks, dim3((uint32_t)ncb), dim3(256), 0, c->stream, aggv, aggf,
                           (uint32_t)nch, totv, totf);
        hipLaunchKernelGGL(k_sfold_carry_top, dim3(1), dim3(1024), 0, c->stream, totv, totf, (uint32_t)ncb,
                           c->fold_round);
        hipLaunchKernelGGL(k_sfold_apply, dim3((uint32_t)nch), dim3(256), 0, c->stream, (const uint64_t*)sk,
                           (const uint64_t*)sv, n, (const uint64_t*)aggv, (const uint32_t*)aggf,
                           (const uint64_t*)totv, (uint64_t*)c->t_keys.p, (uint64_t*)c->t_vals.p, rf);
        HIP_OR_FAIL(c, hipGetLastError());
        if ((s = compact_results(c, n, (const uint64_t*)c->t_keys.p, (const uint64_t*)c->t_vals.p, rf, out_keys,
                                 out_vals, m_out, d_m)) != SS_OK)
            return s;
        return ordered ? order_results(c, out_keys, out_vals, *m_out, params) : SS_OK;
    }
    if (op == SS_MONOID_FIRST || op == SS_MONOID_LAST) {
        // the first / last record of a key is the one at the smallest /
        // largest position: reduce the positions, then fetch the values
        if ((s = ensure(c, c->pos, n * 8)) != SS_OK) return s;
        const uint32_t g = (uint32_t)std::min<uint64_t>((n + 255) / 256, 65536);
        hipLaunchKernelGGL(k_iota, dim3(g), dim3(256), 0, c->stream, (uint64_t*)c->pos.p, n);
        HIP_OR_FAIL(c, hipGetLastError());
        const uint32_t pop = op == SS_MONOID_FIRST ? SS_MONOID_MIN : SS_MONOID_MAX;
        if ((s = run_reduce<1>(c, keys, (const uint64_t*)c->pos.p, n, out_keys, out_vals, m_out, p, pop, d_m)) !=
            SS_OK)
            return s;
        if (m_out) {
            if (*m_out) {
                hipLaunchKernelGGL(k_gather_at, dim3((uint32_t)std::min<uint64_t>((*m_out + 255) / 256, 65536)),
                                   dim3(256), 0, c->stream, out_vals, *m_out, vals, n, (LevelInfo*)c->info.p);
                HIP_OR_FAIL(c, hipGetLastError());
            }
            if (ordered) return order_results(c, out_keys, out_vals, *m_out, params);
            return ss_sync(c);
        }
        // m stays on the device: the gather reads it there
        hipLaunchKernelGGL(k_gather_at_dev, dim3((uint32_t)std::min<uint64_t>((n + 255) / 256, 65536)), dim3(256), 0,
                           c->stream, out_vals, (const uint64_t*)d_m, vals, n, (LevelInfo*)c->info.p);
        HIP_OR_FAIL(c, hipGetLastError());
        return SS_OK;
    }
    if ((s = run_reduce<1>(c, keys, vals, n, out_keys, out_vals, m_out, p, (uint32_t)op, d_m)) != SS_OK) return s;
    return ordered ? order_results(c, out_keys, out_vals, *m_out, params) : SS_OK;
}

ss_status ss_collect_reduce_monoid(ss_ctx* c, const uint64_t* keys, const uint64_t* vals, uint64_t n, int op,
                                   int ordered, uint64_t* out_keys, uint64_t* out_vals, uint64_t* m_out,
                                   const ss_params* params)
{
    Params p;
    ss_status s = check_reduce(c, keys, vals, n, out_keys, out_vals, m_out, params, &p);
    if (s != SS_OK) return s;
    if (op < SS_MONOID_SUM || op > SS_MONOID_AFFINE) return fail(c, SS_EINVAL, "unknown monoid");
    *m_out = 0;
    if (n == 0) return SS_OK;
    if (!vals) return fail(c, SS_EINVAL, "null vals");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    return reduce_call(c, keys, vals, n, op, ordered, out_keys, out_vals, m_out, nullptr, params, p);
}

ss_status ss_collect_reduce_async(ss_ctx* c, const uint64_t* keys, const uint64_t* vals, uint64_t n, int op,
                                  int ordered, uint64_t* out_keys, uint64_t* out_vals, uint64_t* d_m,
                                  const ss_params* params)
{
    if (!c) return SS_EINVAL;
    if (!d_m) return fail(c, SS_EINVAL, "null d_m");
    Params p;
    uint64_t unused = 0;
    ss_status s = check_reduce(c, keys, vals, n, out_keys, out_vals, &unused, params, &p);
    if (s != SS_OK) return s;
    if (op < SS_MONOID_SUM || op > SS_MONOID_AFFINE) return fail(c, SS_EINVAL, "unknown monoid");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    if (n == 0) {
        HIP_OR_FAIL(c, hipMemsetAsync(d_m, 0, 8, c->stream));
        return SS_OK;
    }
    if (!vals) return fail(c, SS_EINVAL, "null vals");
    return reduce_call(c, keys, vals, n, op, ordered, out_keys, out_vals, nullptr, d_m, params, p);
}

ss_status ss_histogram_async(ss_ctx* c, const uint64_t* keys, uint64_t n, int ordered, uint64_t* out_keys,
                             uint64_t* out_counts, uint64_t* d_m, const ss_params* params)
{
    if (!c) return SS_EINVAL;
    if (!d_m) return fail(c, SS_EINVAL, "null d_m");
    Params p;
    uint64_t unused = 0;
    ss_status s = check_reduce(c, keys, nullptr, n, out_keys, out_counts, &unused, params, &p);
    if (s != SS_OK) return s;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    if (n == 0) {
        HIP_OR_FAIL(c, hipMemsetAsync(d_m, 0, 8, c->stream));
        return SS_OK;
    }
    uint64_t m_host = 0;
    if ((s = run_reduce<2>(c, keys, nullptr, n, out_keys, out_counts, ordered ? &m_host : nullptr, p, 0, d_m)) !=
        SS_OK)
        return s;
    return ordered ? order_results(c, out_keys, out_counts, m_host, params) : SS_OK;
}

ss_status ss_batch(ss_ctx* c, const ss_job* jobs, uint64_t njobs, const ss_params* params)
{
    if (!c) return SS_EINVAL;
    if (njobs == 0) return SS_OK;
    if (!jobs) return fail(c, SS_EINVAL, "null jobs");
    if (njobs >= (1ull << 31)) return fail(c, SS_EINVAL, "too many jobs");
    // every job on its own, then no output may overlap any other array
    struct Span {
        uintptr_t a, b;
        bool out;
    };
    std::vector<Span> spans;
    spans.reserve(njobs * 5);
    for (uint64_t i = 0; i < njobs; ++i) {
        const ss_job& J = jobs[i];
        const std::string at = "job " + std::to_string(i) + ": ";
        if (J.op < SS_OP_SEMISORT_EQUAL || J.op > SS_OP_COLLECT_REDUCE) return fail(c, SS_EINVAL, at + "unknown op");
        const bool red = J.op == SS_OP_HISTOGRAM || J.op == SS_OP_COLLECT_REDUCE;
        if (!red && J.val_bytes != 4 && J.val_bytes != 8) return fail(c, SS_EINVAL, at + "val_bytes must be 4 or 8");
        if (J.n >= (1ull << 31)) return fail(c, SS_EINVAL, at + "n must be below 2^31");
        if (red && !J.d_m) return fail(c, SS_EINVAL, at + "null d_m");
        if (red) spans.push_back({(uintptr_t)J.d_m, (uintptr_t)J.d_m + 8, true});
        if (J.n == 0) continue;
        if (!J.keys || !J.out_a || !J.out_b || (J.op != SS_OP_HISTOGRAM && !J.vals))
            return fail(c, SS_EINVAL, at + "null array pointer");
        const uint64_t vb = red ? 8 : J.val_bytes;
        spans.push_back({(uintptr_t)J.keys, (uintptr_t)J.keys + J.n * 8, false});
        if (J.op != SS_OP_HISTOGRAM) spans.push_back({(uintptr_t)J.vals, (uintptr_t)J.vals + J.n * vb, false});
        spans.push_back({(uintptr_t)J.out_a, (uintptr_t)J.out_a + J.n * 8, true});
        spans.push_back({(uintptr_t)J.out_b, (uintptr_t)J.out_b + J.n * vb, true});
    }
    std::sort(spans.begin(), spans.end(), [](const Span& x, const Span& y) { return x.a < y.a; });
    uintptr_t max_end = 0, max_out_end = 0;
    for (const Span& x : spans) {
        if ((x.out && max_end > x.a) || (!x.out && max_out_end > x.a))
            return fail(c, SS_EINVAL, "an output of the batch overlaps another array of the batch");
        max_end = std::max(max_end, x.b);
        if (x.out) max_out_end = std::max(max_out_end, x.b);
    }
    Params p;
    ss_status s = resolve_params(c, params, &p);
    if (s != SS_OK) return s;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");

    // groups: semisort_= and semisort_< by value width, histogram, collect-reduce
    constexpr int kGroups = 6;
    auto group_of = [](const ss_job& J) {
        switch (J.op) {
        case SS_OP_SEMISORT_EQUAL: return J.val_bytes == 8 ? 1 : 0;
        case SS_OP_SEMISORT_LESS: return J.val_bytes == 8 ? 3 : 2;
        case SS_OP_HISTOGRAM: return 4;
        default: return 5;
        }
    };
    std::vector<uint32_t> packed[kGroups], direct;
    for (uint64_t i = 0; i < njobs; ++i) {
        const ss_job& J = jobs[i];
        if (J.n == 0) {
            if (J.op == SS_OP_HISTOGRAM || J.op == SS_OP_COLLECT_REDUCE)
                HIP_OR_FAIL(c, hipMemsetAsync(J.d_m, 0, 8, c->stream));
            continue;
        }
        if (J.n <= SS_BATCH_PACK_MAX) packed[group_of(J)].push_back((uint32_t)i);
        else direct.push_back((uint32_t)i);
    }
    // large jobs one by one on their own arrays, as the single calls run them
    for (uint32_t i : direct) {
        const ss_job& J = jobs[i];
        const uint64_t offs[2] = {0, J.n};
        Params q = p;
        switch (J.op) {
        case SS_OP_SEMISORT_EQUAL:
        case SS_OP_SEMISORT_LESS:
            if (J.op == SS_OP_SEMISORT_LESS) {
                q.mode = 2;
                default_tiles(c, params, &q, 32768u, 65536u);
            } else {
                default_tiles(c, params, &q, 32768u, 16384u);
            }
            s = J.val_bytes == 8
                    ? run_semisort<uint64_t>(c, J.keys, J.vals, offs, 1, (uint64_t*)J.out_a, J.out_b, q)
                    : run_semisort<uint32_t>(c, J.keys, J.vals, offs, 1, (uint64_t*)J.out_a, J.out_b, q);
            break;
        case SS_OP_HISTOGRAM:
            s = run_reduce<2>(c, J.keys, nullptr, J.n, (uint64_t*)J.out_a, (uint64_t*)J.out_b, nullptr, p, 0, J.d_m);
            break;
        default:
            s = run_reduce<1>(c, J.keys, (const uint64_t*)J.vals, J.n, (uint64_t*)J.out_a, (uint64_t*)J.out_b,
                              nullptr, p, 0, J.d_m);
            break;
        }
        if (s != SS_OK) return s;
    }
    // the packed job tables of every group, staged and copied at once
    uint64_t ntab = 0;
    for (int g = 0; g < kGroups; ++g) ntab += packed[g].size();
    if (!ntab) return SS_OK;
    if ((s = stage_wait(c)) != SS_OK) return s;
    if ((s = ensure_pinned(c, (void**)&c->pack_stage, &c->pack_stage_cap, ntab * sizeof(PackJob))) != SS_OK) return s;
    if ((s = ensure(c, c->pack_tab, ntab * sizeof(PackJob))) != SS_OK) return s;
    uint64_t tab0[kGroups], total[kGroups];
    std::vector<uint64_t> offs[kGroups];
    {
        uint64_t t = 0;
        for (int g = 0; g < kGroups; ++g) {
            tab0[g] = t;
            offs[g].assign(1, 0);
            for (uint32_t i : packed[g]) {
                const ss_job& J = jobs[i];
                PackJob& e = c->pack_stage[t++];
                e.keys = J.keys;
                e.vals = J.vals;
                e.out_a = J.out_a;
                e.out_b = J.out_b;
                e.d_m = J.d_m;
                e.off = offs[g].back();
                e.n = J.n;
                offs[g].push_back(e.off + J.n);
            }
            total[g] = offs[g].back();
        }
    }
    HIP_OR_FAIL(c, hipMemcpyAsync(c->pack_tab.p, c->pack_stage, ntab * sizeof(PackJob), hipMemcpyHostToDevice,
                                  c->stream));
    if ((s = stage_mark(c)) != SS_OK) return s;
    const PackJob* dtab = (const PackJob*)c->pack_tab.p;
    for (int g = 0; g < kGroups; ++g) {
        const uint32_t nj = (uint32_t)packed[g].size();
        if (!nj) continue;
        const uint64_t tot = total[g];
        const bool red = g >= 4;
        const uint32_t vb = red || (g & 1) ? 8 : 4;
        if ((s = ensure(c, c->pk_k, tot * 8)) != SS_OK) return s;
        if (g != 4 && (s = ensure(c, c->pk_v, tot * vb)) != SS_OK) return s;
        if ((s = ensure(c, c->po_k, tot * 8)) != SS_OK) return s;
        if ((s = ensure(c, c->po_v, tot * vb)) != SS_OK) return s;
        const PackJob* tab = dtab + tab0[g];
        const uint32_t grid = (uint32_t)((tot + kPackChunk - 1) / kPackChunk);
        uint64_t* pk = (uint64_t*)c->pk_k.p;
        uint64_t* ok = (uint64_t*)c->po_k.p;
        if (vb == 8)
            hipLaunchKernelGGL((k_pack_gather<uint64_t>), dim3(grid), dim3(256), 0, c->stream, tab, nj, tot, pk,
                               g == 4 ? nullptr : (uint64_t*)c->pk_v.p);
        else
            hipLaunchKernelGGL((k_pack_gather<uint32_t>), dim3(grid), dim3(256), 0, c->stream, tab, nj, tot, pk,
                               (uint32_t*)c->pk_v.p);
        HIP_OR_FAIL(c, hipGetLastError());
        if (!red) {
            Params q = p;
            if (g >= 2) q.mode = 2;
            s = vb == 8 ? run_semisort<uint64_t>(c, pk, c->pk_v.p, offs[g].data(), nj, ok, c->po_v.p, q)
                        : run_semisort<uint32_t>(c, pk, c->pk_v.p, offs[g].data(), nj, ok, c->po_v.p, q);
            if (s != SS_OK) return s;
            if (vb == 8)
                hipLaunchKernelGGL((k_pack_scatter<uint64_t>), dim3(grid), dim3(256), 0, c->stream, tab, nj, tot, ok,
                                   (const uint64_t*)c->po_v.p);
            else
                hipLaunchKernelGGL((k_pack_scatter<uint32_t>), dim3(grid), dim3(256), 0, c->stream, tab, nj, tot, ok,
                                   (const uint32_t*)c->po_v.p);
        } else {
            s = g == 4 ? run_reduce_multi<2>(c, pk, nullptr, offs[g].data(), nj, ok, (uint64_t*)c->po_v.p, nullptr, p,
                                             0, nullptr)
                       : run_reduce_multi<1>(c, pk, (const uint64_t*)c->pk_v.p, offs[g].data(), nj, ok,
                                             (uint64_t*)c->po_v.p, nullptr, p, 0, nullptr);
            if (s != SS_OK) return s;
            // every job's pairs are a contiguous run of the packed pairs
            if ((s = ensure(c, c->pack_rank, (size_t)(nj + 1) * 8)) != SS_OK) return s;
            const uint64_t nblk = (tot + kFlagBlock - 1) / kFlagBlock;
            const uint32_t* ccnt = (const uint32_t*)c->bcnt.p;
            const uint32_t* boff = ccnt + nblk * (kFlagBlock / kFlagChunk);
            uint64_t* rank = (uint64_t*)c->pack_rank.p;
            hipLaunchKernelGGL(k_inst_ranks, dim3(nj + 1), dim3(256), 0, c->stream, (const uint8_t*)c->rflag.p, ccnt,
                               boff, tab, nj, (const unsigned long long*)c->mdev.p, rank);
            hipLaunchKernelGGL(k_inst_m, dim3((nj + 255) / 256), dim3(256), 0, c->stream, tab, nj,
                               (const uint64_t*)rank);
            hipLaunchKernelGGL(k_pack_scatter_red, dim3(grid), dim3(256), 0, c->stream, tab, nj,
                               (const uint64_t*)rank, (const uint64_t*)ok, (const uint64_t*)c->po_v.p);
        }
        HIP_OR_FAIL(c, hipGetLastError());
    }
    return SS_OK;
}

ss_status ss_collect_reduce_ordered(ss_ctx* c, const uint64_t* keys, const uint64_t* vals, uint64_t n,
                                    uint64_t* out_keys, uint64_t* out_sums, uint64_t* m_out, const ss_params* params)
{
    ss_status s = ss_collect_reduce(c, keys, vals, n, out_keys, out_sums, m_out, params);
    if (s != SS_OK) return s;
    return order_results(c, out_keys, out_sums, *m_out, params);
}

ss_status ss_histogram_ordered(ss_ctx* c, const uint64_t* keys, uint64_t n, uint64_t* out_keys,
                               uint64_t* out_counts, uint64_t* m_out, const ss_params* params)
{
    ss_status s = ss_histogram(c, keys, n, out_keys, out_counts, m_out, params);
    if (s != SS_OK) return s;
    return order_results(c, out_keys, out_counts, *m_out, params);
}

// ---------------------------------------------------------------- caller monoids

ss_status ss_monoid_compile(ss_ctx* c, const char* source, ss_user_monoid** out)
{
    if (!c) return SS_EINVAL;
    if (!source || !out) return fail(c, SS_EINVAL, "null source or out");
    *out = nullptr;
    // the caller's definitions, then the fold kernels that use them; #line
    // makes compiler messages count the caller's lines from 1
    const std::string full = std::string(kUserFoldPrelude) + "#line 1 \"monoid\"\n" + source + "\n#line 1 \"ss_fold\"\n" +
                             kUserFoldKernels;
    hiprtcProgram prog = nullptr;
    if (hiprtcCreateProgram(&prog, full.c_str(), "ss_monoid.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return fail(c, SS_EHIP, "hiprtcCreateProgram");
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops"};
    if (hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts) != HIPRTC_SUCCESS) {
        size_t ls = 0;
        std::string log;
        if (hiprtcGetProgramLogSize(prog, &ls) == HIPRTC_SUCCESS && ls) {
            log.resize(ls);
            if (hiprtcGetProgramLog(prog, &log[0]) != HIPRTC_SUCCESS) log.clear();
        }
        hiprtcDestroyProgram(&prog);
        return fail(c, SS_EINVAL, "the monoid source does not compile: " + log);
    }
    size_t cs = 0;
    std::vector<char> code;
    if (hiprtcGetCodeSize(prog, &cs) == HIPRTC_SUCCESS && cs) {
        code.resize(cs);
        if (hiprtcGetCode(prog, code.data()) != HIPRTC_SUCCESS) code.clear();
    }
    hiprtcDestroyProgram(&prog);
    if (code.empty()) return fail(c, SS_EHIP, "hiprtcGetCode");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    ss_user_monoid* m = new (std::nothrow) ss_user_monoid;
    if (!m) return fail(c, SS_ENOMEM, "monoid");
    m->device = c->device;
    if (hipModuleLoadData(&m->mod, code.data()) != hipSuccess) {
        delete m;
        return fail(c, SS_EHIP, "hipModuleLoadData");
    }
    if (hipModuleGetFunction(&m->aggr, m->mod, "ss_fold_aggr") != hipSuccess ||
        hipModuleGetFunction(&m->carry_blocks, m->mod, "ss_fold_carry_blocks") != hipSuccess ||
        hipModuleGetFunction(&m->carry_top, m->mod, "ss_fold_carry_top") != hipSuccess ||
        hipModuleGetFunction(&m->apply, m->mod, "ss_fold_apply") != hipSuccess) {
        (void)hipModuleUnload(m->mod);
        delete m;
        return fail(c, SS_EHIP, "hipModuleGetFunction");
    }
    *out = m;
    return SS_OK;
}

ss_status ss_monoid_destroy(ss_user_monoid* m)
{
    if (!m) return SS_EINVAL;
    (void)hipSetDevice(m->device);
    (void)hipModuleUnload(m->mod);
    delete m;
    return SS_OK;
}

ss_status ss_collect_reduce_user(ss_ctx* c, const ss_user_monoid* mo, const uint64_t* keys, const void* vals,
                                 uint32_t vb, uint64_t n, int ordered, uint64_t* out_keys, uint64_t* out_vals,
                                 uint64_t* m_out, const ss_params* params)
{
    if (!c) return SS_EINVAL;
    if (!mo) return fail(c, SS_EINVAL, "null monoid");
    if (mo->device != c->device) return fail(c, SS_EINVAL, "the monoid was compiled for another device");
    if (vb != 4 && vb != 8) return fail(c, SS_EINVAL, "val_bytes must be 4 or 8");
    Params p;
    ss_status s = check_reduce(c, keys, nullptr, n, out_keys, out_vals, m_out, params, &p);
    if (s != SS_OK) return s;
    *m_out = 0;
    if (n == 0) return SS_OK;
    if (!vals) return fail(c, SS_EINVAL, "null vals");
    if (overlaps(out_keys, n * 8, vals, n * vb) || overlaps(out_vals, n * 8, vals, n * vb))
        return fail(c, SS_EINVAL, "outputs overlap inputs");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SS_EHIP, "hipSetDevice");
    // a stable semisort_= makes every key's records contiguous and in input
    // order; the fold then runs over positions
    Params q = p;
    default_tiles(c, params, &q, 32768u, 16384u);
    if ((s = ensure(c, c->tr_keys, n * 8)) != SS_OK) return s;
    if ((s = ensure(c, c->tr_sorted, n * vb)) != SS_OK) return s;
    uint64_t* sk = (uint64_t*)c->tr_keys.p;
    void* sv = c->tr_sorted.p;
    const uint64_t so[2] = {0, n};
    if ((s = vb == 8 ? run_semisort<uint64_t>(c, keys, vals, so, 1, sk, sv, q)
                     : run_semisort<uint32_t>(c, keys, vals, so, 1, sk, sv, q)) != SS_OK)
        return s;
    const uint64_t nblk = (n + kFlagBlock - 1) / kFlagBlock;
    const uint64_t nch = (n + kFoldChunk - 1) / kFoldChunk;
    const uint64_t ncb = (nch + 255) / 256;
    if ((s = ensure(c, c->t_keys, n * 8)) != SS_OK) return s;
    if ((s = ensure(c, c->t_vals, n * 8)) != SS_OK) return s;
    if ((s = ensure(c, c->rflag, nblk * kFlagBlock)) != SS_OK) return s;
    if ((s = ensure(c, c->bcnt, (nblk * (kFlagBlock / kFlagChunk) + nblk) * 4)) != SS_OK) return s;
    if ((s = ensure(c, c->mdev, 8)) != SS_OK) return s;
    if ((s = ensure(c, c->pos, (nch + ncb) * 12)) != SS_OK) return s;
    // 8 bytes per element of the monoid (its type is at most 8 bytes)
    void* aggv = c->pos.p;
    void* totv = (char*)aggv + nch * 8;
    uint32_t* aggf = (uint32_t*)((char*)totv + ncb * 8);
    uint32_t* totf = aggf + nch;
    uint8_t* rf = (uint8_t*)c->rflag.p;
    HIP_OR_FAIL(c, hipMemsetAsync(rf, 0, nblk * kFlagBlock, c->stream));
    const uint64_t* ck = sk;
    const void* cv = sv;
    uint32_t vbk = vb;
    uint64_t nk = n;
    uint32_t nchk = (uint32_t)nch, ncbk = (uint32_t)ncb, rb = c->fold_round;
    uint64_t* rk = (uint64_t*)c->t_keys.p;
    uint64_t* rv = (uint64_t*)c->t_vals.p;
    {
        void* a[] = {&ck, &cv, &vbk, &nk, &aggv, &aggf};
        HIP_OR_FAIL(c, hipModuleLaunchKernel(mo->aggr, nchk, 1, 1, 256, 1, 1, 0, c->stream, a, nullptr));
    }
    {
        void* a[] = {&aggv, &aggf, &nchk, &totv, &totf};
        HIP_OR_FAIL(c, hipModuleLaunchKernel(mo->carry_blocks, ncbk, 1, 1, 256, 1, 1, 0, c->stream, a, nullptr));
    }
    {
        void* a[] = {&totv, &totf, &ncbk, &rb};
        HIP_OR_FAIL(c, hipModuleLaunchKernel(mo->carry_top, 1, 1, 1, 1024, 1, 1, 0, c->stream, a, nullptr));
    }
    {
        void* a[] = {&ck, &cv, &vbk, &nk, &aggv, &aggf, &totv, &rk, &rv, &rf};
        HIP_OR_FAIL(c, hipModuleLaunchKernel(mo->apply, nchk, 1, 1, 256, 1, 1, 0, c->stream, a, nullptr));
    }
    if ((s = compact_results(c, n, (const uint64_t*)rk, (const uint64_t*)rv, rf, out_keys, out_vals, m_out)) != SS_OK)
        return s;
    return ordered ? order_results(c, out_keys, out_vals, *m_out, params) : SS_OK;
}

}  // extern "C"
