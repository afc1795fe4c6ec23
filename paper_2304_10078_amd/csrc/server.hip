// Request server of libsemisort_hip.so (declared in include/semisort.h).
//
// Group-by requests (semisort_=, semisort_<, histogram, collect-reduce) are
// queued on submission and served by `lanes` worker threads, each driving its
// own context on its own HIP stream, so requests on different lanes run on
// the device at the same time.  A free lane takes the oldest request whose
// workspace fits in the HBM budget; small semisort_= requests waiting behind
// it with the same value width are packed into the lane's buffers and run as
// one batched call (continuous batching): every instance of a batch gives the
// result it gives alone.  Completion is observed on the host after the lane's
// stream drains; latency runs from arrival to that moment.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "semisort.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Ticket {
    ss_request req;
    double arrival = 0.0;
    double done_at = 0.0;
    std::atomic<int> done{0};
    ss_status status = SS_OK;
    uint64_t m = 0;
};

struct Lane {
    int index = 0;
    hipStream_t stream = nullptr;
    ss_ctx* ctx = nullptr;
    // packing buffers: keys and values in, keys and values out
    void* pk_in = nullptr;
    void* pv_in = nullptr;
    void* pk_out = nullptr;
    void* pv_out = nullptr;
    uint64_t reserved = 0;  // bytes this lane may hold (workspace estimate, packing buffers)
    std::thread th;
};

}  // namespace

struct ss_server {
    int device = 0;
    ss_server_config cfg;
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;       // work arrived / memory freed / stop
    std::condition_variable idle_cv;  // a request completed
    std::deque<uint64_t> queue;       // ticket ids in arrival order
    std::deque<Ticket> tickets;       // stable addresses; index = ticket id
    std::vector<Lane> lanes;
    uint64_t reserved = 0;            // sum over lanes
    uint64_t peak_reserved = 0;
    uint64_t in_flight = 0;
    uint64_t completed = 0, batches = 0, packed = 0;
    bool stop = false;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

bool is_semisort(int op) { return op == SS_OP_SEMISORT_EQUAL || op == SS_OP_SEMISORT_LESS; }

// Device workspace a context needs for a request of n records (the
// temporary array, bucket ids and, for collect-reduce, the result flags),
// plus a fixed allowance for tables and work lists.
uint64_t workspace_estimate(const ss_request& r)
{
    const uint64_t vb = r.op == SS_OP_HISTOGRAM || r.op == SS_OP_COLLECT_REDUCE ? 8 : r.val_bytes;
    uint64_t b = r.n * (8 + vb) + 2 * r.n;
    if (!is_semisort(r.op)) b += r.n + 4 * (r.n / 65536 + 1);
    return b + (64ull << 20);
}

ss_status run_one(const ss_params* prm, Lane& L, Ticket& t)
{
    const ss_request& r = t.req;
    ss_status s;
    switch (r.op) {
    case SS_OP_SEMISORT_EQUAL:
        s = ss_semisort_equal(L.ctx, r.keys, r.vals, r.val_bytes, r.n, (uint64_t*)r.out_a, r.out_b, prm);
        break;
    case SS_OP_SEMISORT_LESS:
        s = ss_semisort_less(L.ctx, r.keys, r.vals, r.val_bytes, r.n, (uint64_t*)r.out_a, r.out_b, prm);
        break;
    case SS_OP_HISTOGRAM:
        s = ss_histogram(L.ctx, r.keys, r.n, (uint64_t*)r.out_a, (uint64_t*)r.out_b, &t.m, prm);
        break;
    default:
        s = ss_collect_reduce(L.ctx, r.keys, (const uint64_t*)r.vals, r.n, (uint64_t*)r.out_a,
                              (uint64_t*)r.out_b, &t.m, prm);
        break;
    }
    if (s != SS_OK) return s;
    return ss_sync(L.ctx);
}

// Packed semisort_= of several requests: copy in, one batched call, copy out.
ss_status run_packed(ss_server* S, Lane& L, const std::vector<Ticket*>& group)
{
    const uint32_t vb = group[0]->req.val_bytes;
    std::vector<uint64_t> offs(group.size() + 1, 0);
    for (size_t i = 0; i < group.size(); ++i) offs[i + 1] = offs[i] + group[i]->req.n;
    for (size_t i = 0; i < group.size(); ++i) {
        const ss_request& r = group[i]->req;
        if (hipMemcpyAsync((uint64_t*)L.pk_in + offs[i], r.keys, r.n * 8, hipMemcpyDeviceToDevice, L.stream) !=
                hipSuccess ||
            hipMemcpyAsync((char*)L.pv_in + offs[i] * vb, r.vals, r.n * vb, hipMemcpyDeviceToDevice, L.stream) !=
                hipSuccess)
            return SS_EHIP;
    }
    ss_status s = ss_semisort_equal_batch(L.ctx, (const uint64_t*)L.pk_in, L.pv_in, vb, offs.data(), group.size(),
                                          (uint64_t*)L.pk_out, L.pv_out, &S->cfg.params);
    if (s != SS_OK) return s;
    for (size_t i = 0; i < group.size(); ++i) {
        const ss_request& r = group[i]->req;
        if (hipMemcpyAsync(r.out_a, (uint64_t*)L.pk_out + offs[i], r.n * 8, hipMemcpyDeviceToDevice, L.stream) !=
                hipSuccess ||
            hipMemcpyAsync(r.out_b, (char*)L.pv_out + offs[i] * vb, r.n * vb, hipMemcpyDeviceToDevice, L.stream) !=
                hipSuccess)
            return SS_EHIP;
    }
    return ss_sync(L.ctx);
}

void worker(ss_server* S, int li)
{
    Lane& L = S->lanes[li];
    (void)hipSetDevice(S->device);
    const uint64_t pack_cap = S->cfg.batch_records;
    for (;;) {
        std::vector<Ticket*> group;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                if (S->stop) return;
                // the oldest request that fits in the budget with this lane's share
                size_t pick = S->queue.size();
                uint64_t need = 0;
                for (size_t qi = 0; qi < S->queue.size(); ++qi) {
                    Ticket& t = S->tickets[S->queue[qi]];
                    const uint64_t est = std::max<uint64_t>(L.reserved, workspace_estimate(t.req));
                    if (S->reserved - L.reserved + est <= S->cfg.hbm_budget) {
                        pick = qi;
                        need = est;
                        break;
                    }
                }
                if (pick < S->queue.size()) {
                    Ticket* head = &S->tickets[S->queue[pick]];
                    S->queue.erase(S->queue.begin() + (long)pick);
                    group.push_back(head);
                    S->reserved += need - L.reserved;
                    L.reserved = need;
                    S->peak_reserved = std::max(S->peak_reserved, S->reserved);
                    // continuous batching: small semisort_= requests of the same
                    // value width that are already waiting join this call
                    const ss_request& h = head->req;
                    if (h.op == SS_OP_SEMISORT_EQUAL && h.n <= S->cfg.pack_max_records && L.pk_in) {
                        // (each joins only if the workspace for the whole batch fits)
                        ss_request all = h;
                        for (size_t qi = 0; qi < S->queue.size();) {
                            Ticket& t = S->tickets[S->queue[qi]];
                            ss_request more = all;
                            more.n = all.n + t.req.n;
                            const uint64_t est = std::max<uint64_t>(L.reserved, workspace_estimate(more));
                            if (t.req.op == SS_OP_SEMISORT_EQUAL && t.req.val_bytes == h.val_bytes &&
                                t.req.n <= S->cfg.pack_max_records && more.n <= pack_cap &&
                                S->reserved - L.reserved + est <= S->cfg.hbm_budget) {
                                all.n = more.n;
                                S->reserved += est - L.reserved;
                                L.reserved = est;
                                S->peak_reserved = std::max(S->peak_reserved, S->reserved);
                                group.push_back(&t);
                                S->queue.erase(S->queue.begin() + (long)qi);
                            } else {
                                ++qi;
                            }
                        }
                    }
                    break;
                }
                // nothing fits: an idle lane gives its workspace back first
                // (it keeps its packing buffers)
                const uint64_t pack_bytes = L.pk_in ? 4 * pack_cap * 8 : 0;
                if (L.reserved > pack_bytes && !S->queue.empty()) {
                    ss_ctx* fresh = nullptr;
                    if (ss_create(S->device, L.stream, &fresh) == SS_OK) {
                        (void)ss_destroy(L.ctx);
                        L.ctx = fresh;
                        S->reserved -= L.reserved - pack_bytes;
                        L.reserved = pack_bytes;
                        S->cv.notify_all();  // other idle lanes look again (and give back too)
                        continue;
                    }
                }
                S->cv.wait(lk);
            }
        }
        ss_status st;
        if (group.size() == 1) st = run_one(&S->cfg.params, L, *group[0]);
        else st = run_packed(S, L, group);
        const double t_done = S->now();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (Ticket* t : group) {
                t->status = st;
                t->done_at = t_done;
                t->done.store(1);
            }
            S->completed += group.size();
            S->in_flight -= group.size();
            S->batches += 1;
            if (group.size() > 1) S->packed += group.size();
            // what the context really holds now
            size_t ws = 0;
            if (ss_workspace_bytes(L.ctx, &ws) == SS_OK) {
                const uint64_t pack_bytes = L.pk_in ? 4 * pack_cap * 8 : 0;
                const uint64_t held = (uint64_t)ws + pack_bytes;
                if (held > L.reserved) {
                    S->reserved += held - L.reserved;
                    L.reserved = held;
                    S->peak_reserved = std::max(S->peak_reserved, S->reserved);
                }
            }
        }
        S->cv.notify_all();
        S->idle_cv.notify_all();
    }
}

}  // namespace

extern "C" {

ss_status ss_server_default_config(ss_server_config* c)
{
    if (!c) return SS_EINVAL;
    c->lanes = 4;
    c->pack_max_records = 1u << 20;
    c->batch_records = 1ull << 24;
    c->hbm_budget = 200ull << 30;
    return ss_default_params(&c->params);
}

ss_status ss_server_create(int device, const ss_server_config* cfg, ss_server** out)
{
    if (!out) return SS_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SS_EINVAL;
    ss_server_config c;
    if (cfg) c = *cfg;
    else ss_server_default_config(&c);
    if (c.lanes < 1 || c.lanes > 16) return SS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return SS_EHIP;
    ss_server* S = new (std::nothrow) ss_server();
    if (!S) return SS_ENOMEM;
    S->device = device;
    S->cfg = c;
    S->t0 = Clock::now();
    S->lanes.resize(c.lanes);
    ss_status st = SS_OK;
    for (uint32_t i = 0; i < c.lanes && st == SS_OK; ++i) {
        Lane& L = S->lanes[i];
        L.index = (int)i;
        if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess) {
            st = SS_EHIP;
            break;
        }
        if ((st = ss_create(device, L.stream, &L.ctx)) != SS_OK) break;
        if (c.pack_max_records && c.batch_records) {
            const size_t kb = c.batch_records * 8;
            if (hipMalloc(&L.pk_in, kb) != hipSuccess || hipMalloc(&L.pv_in, kb) != hipSuccess ||
                hipMalloc(&L.pk_out, kb) != hipSuccess || hipMalloc(&L.pv_out, kb) != hipSuccess) {
                st = SS_ENOMEM;
                break;
            }
            L.reserved = 4 * kb;
            S->reserved += L.reserved;
        }
    }
    if (st == SS_OK && S->reserved > c.hbm_budget) st = SS_EINVAL;  // packing buffers alone exceed the budget
    if (st != SS_OK) {
        for (Lane& L : S->lanes) {
            if (L.ctx) ss_destroy(L.ctx);
            for (void* p : {L.pk_in, L.pv_in, L.pk_out, L.pv_out})
                if (p) (void)hipFree(p);
            if (L.stream) (void)hipStreamDestroy(L.stream);
        }
        delete S;
        return st;
    }
    S->peak_reserved = S->reserved;
    for (uint32_t i = 0; i < c.lanes; ++i) S->lanes[i].th = std::thread(worker, S, (int)i);
    *out = S;
    return SS_OK;
}

double ss_server_now(ss_server* S)
{
    return S ? S->now() : 0.0;
}

ss_status ss_server_submit(ss_server* S, const ss_request* r, double arrival_s, uint64_t* ticket)
{
    if (!S || !r || !ticket) return SS_EINVAL;
    if (r->op < SS_OP_SEMISORT_EQUAL || r->op > SS_OP_COLLECT_REDUCE) return SS_EINVAL;
    if (is_semisort(r->op) && r->val_bytes != 4 && r->val_bytes != 8) return SS_EINVAL;
    if (r->n >= (1ull << 31)) return SS_EINVAL;
    if (r->n && (!r->keys || !r->out_a || !r->out_b || (r->op != SS_OP_HISTOGRAM && !r->vals))) return SS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return SS_EINVAL;
    // a request that cannot fit even with every lane's workspace given back
    uint64_t pack_total = 0;
    for (const Lane& L : S->lanes)
        if (L.pk_in) pack_total += 4 * S->cfg.batch_records * 8;
    if (r->n && workspace_estimate(*r) + pack_total > S->cfg.hbm_budget) return SS_ENOMEM;
    S->tickets.emplace_back();
    Ticket& t = S->tickets.back();
    t.req = *r;
    t.arrival = arrival_s > 0.0 ? arrival_s : S->now();
    const uint64_t id = S->tickets.size() - 1;
    *ticket = id;
    if (r->n == 0) {
        t.done_at = S->now();
        t.done.store(1);
        S->completed += 1;
        return SS_OK;
    }
    S->queue.push_back(id);
    S->in_flight += 1;
    S->cv.notify_one();
    return SS_OK;
}

ss_status ss_server_poll(ss_server* S, uint64_t ticket, int* done, ss_status* result, double* latency_s,
                         uint64_t* m)
{
    if (!S || !done) return SS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (ticket >= S->tickets.size()) return SS_EINVAL;
    Ticket& t = S->tickets[ticket];
    *done = t.done.load();
    if (*done) {
        if (result) *result = t.status;
        if (latency_s) *latency_s = t.done_at - t.arrival;
        if (m) *m = t.m;
    }
    return SS_OK;
}

ss_status ss_server_drain(ss_server* S)
{
    if (!S) return SS_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    S->idle_cv.wait(lk, [&] { return S->in_flight == 0; });
    return SS_OK;
}

ss_status ss_server_stats(ss_server* S, uint64_t* completed, uint64_t* calls, uint64_t* packed,
                          uint64_t* peak_reserved)
{
    if (!S) return SS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (completed) *completed = S->completed;
    if (calls) *calls = S->batches;
    if (packed) *packed = S->packed;
    if (peak_reserved) *peak_reserved = S->peak_reserved;
    return SS_OK;
}

ss_status ss_server_destroy(ss_server* S)
{
    if (!S) return SS_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    for (Lane& L : S->lanes)
        if (L.th.joinable()) L.th.join();
    (void)hipSetDevice(S->device);
    for (Lane& L : S->lanes) {
        if (L.ctx) ss_destroy(L.ctx);
        for (void* p : {L.pk_in, L.pv_in, L.pk_out, L.pv_out})
            if (p) (void)hipFree(p);
        if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    delete S;
    return SS_OK;
}

}  // extern "C"
