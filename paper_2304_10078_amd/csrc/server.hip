// Request server of libsemisort_hip.so (declared in include/semisort.h).
//
// Group-by requests (semisort_=, semisort_<, histogram, collect-reduce) are
// queued on submission and served by `lanes` worker threads, each driving its
// own context on its own HIP stream, so requests on different lanes run on
// the device at the same time.  A free lane takes the oldest request that
// fits in the HBM budget, and the small requests of any operation waiting
// behind it join the same call (continuous batching): the lane runs them as
// one ss_batch, which packs them into one launch chain per operation and
// level, and every request gets the result it gets alone.  The budget counts
// the arrays of the requests being served (inputs and outputs) and every
// lane's workspace: what it holds plus an upper bound of what the call may
// add (the planning bound of ss_workspace_bytes), so the total stays within
// the budget.  Completion is observed on the host after the lane's stream
// drains; latency runs from arrival to that moment.
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

// Requests one lane call takes at most (the device array of group counts).
constexpr uint32_t kMaxBatchJobs = 4096;

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
    uint64_t* d_m = nullptr;  // device: m of every reduction of the lane's call
    uint64_t* h_m = nullptr;  // pinned copy
    uint64_t ws = 0;          // bytes charged for the lane's workspace
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
    uint64_t ws_charged = 0;          // sum of the lanes' workspace charges
    uint64_t io_charged = 0;          // inputs and outputs of the requests being served
    uint64_t peak_reserved = 0;
    uint64_t in_flight = 0;
    uint64_t completed = 0, batches = 0, packed = 0;
    bool stop = false;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    uint64_t reserved() const { return ws_charged + io_charged; }
};

namespace {

bool is_reduce(int op) { return op == SS_OP_HISTOGRAM || op == SS_OP_COLLECT_REDUCE; }

uint64_t value_bytes(const ss_request& r) { return is_reduce(r.op) ? 8 : r.val_bytes; }

// Device memory of a request's own arrays: keys and values in, both outputs.
uint64_t io_bytes(const ss_request& r)
{
    const uint64_t vb = value_bytes(r);
    return r.n * (8 + (r.op == SS_OP_HISTOGRAM ? 0 : vb) + 8 + vb);
}

// Upper bound of the workspace one ss_batch call over `group` adds to a
// context: the planning bound of every operation group's packed total (the
// groups share the buffers, so the sum bounds their largest), packing
// buffers of 2 x (8 + value bytes) per packed record twice, and the job table.
uint64_t batch_bound(const std::vector<Ticket*>& group, const ss_params* prm)
{
    uint64_t tot[6] = {}, big = 0, njobs = group.size();
    for (const Ticket* t : group) {
        const ss_request& r = t->req;
        int g = r.op == SS_OP_HISTOGRAM ? 4 : r.op == SS_OP_COLLECT_REDUCE ? 5 : 2 * r.op + (r.val_bytes == 8);
        if (r.n > SS_BATCH_PACK_MAX) {
            size_t b = 0;
            if (ss_workspace_bytes(r.op, r.n, (uint32_t)value_bytes(r), prm, &b) == SS_OK) big += b;
        } else {
            tot[g] += r.n;
        }
    }
    uint64_t b = big + njobs * 64 + (64ull << 10);
    for (int g = 0; g < 6; ++g) {
        if (!tot[g]) continue;
        const int op = g == 4 ? SS_OP_HISTOGRAM : g == 5 ? SS_OP_COLLECT_REDUCE : g / 2;
        const uint32_t vb = g >= 4 || (g & 1) ? 8 : 4;
        size_t w = 0;
        if (ss_workspace_bytes(op, tot[g], vb, prm, &w) == SS_OK) b += w;
        b += 2 * tot[g] * (8 + vb) + 512;
    }
    return b;
}

// One call for the whole group: small requests are packed by ss_batch, the
// counts of the reductions come back through the lane's device array.
ss_status run_group(ss_server* S, Lane& L, const std::vector<Ticket*>& group)
{
    std::vector<ss_job> jobs(group.size());
    for (size_t i = 0; i < group.size(); ++i) {
        const ss_request& r = group[i]->req;
        ss_job& j = jobs[i];
        j.op = r.op;
        j.val_bytes = r.val_bytes;
        j.n = r.n;
        j.keys = r.keys;
        j.vals = r.vals;
        j.out_a = r.out_a;
        j.out_b = r.out_b;
        j.d_m = is_reduce(r.op) ? L.d_m + i : nullptr;
    }
    ss_status s = ss_batch(L.ctx, jobs.data(), jobs.size(), &S->cfg.params);
    if (s != SS_OK) return s;
    if (hipMemcpyAsync(L.h_m, L.d_m, group.size() * 8, hipMemcpyDeviceToHost, L.stream) != hipSuccess)
        return SS_EHIP;
    if ((s = ss_sync(L.ctx)) != SS_OK) return s;
    for (size_t i = 0; i < group.size(); ++i)
        if (is_reduce(group[i]->req.op)) group[i]->m = L.h_m[i];
    return SS_OK;
}

void worker(ss_server* S, int li)
{
    Lane& L = S->lanes[li];
    (void)hipSetDevice(S->device);
    const uint64_t budget = S->cfg.hbm_budget;
    for (;;) {
        std::vector<Ticket*> group;
        uint64_t group_io = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                if (S->stop) return;
                // The oldest request whose arrays and workspace fit in the
                // budget beside everything else being served.  The lane is
                // charged its current workspace plus the bound of what the
                // call may add, so the total never passes the budget.
                size_t pick = S->queue.size();
                uint64_t charge = 0;
                for (size_t qi = 0; qi < S->queue.size(); ++qi) {
                    Ticket& t = S->tickets[S->queue[qi]];
                    const uint64_t need = L.ws + batch_bound({&t}, &S->cfg.params);
                    if (S->reserved() - L.ws + need + io_bytes(t.req) <= budget) {
                        pick = qi;
                        charge = need;
                        break;
                    }
                }
                if (pick < S->queue.size()) {
                    Ticket* head = &S->tickets[S->queue[pick]];
                    S->queue.erase(S->queue.begin() + (long)pick);
                    group.push_back(head);
                    group_io = io_bytes(head->req);
                    // continuous batching: small requests already waiting join
                    // this call while the batch and the budget allow
                    uint64_t recs = head->req.n;
                    if (head->req.n <= S->cfg.pack_max_records) {
                        for (size_t qi = 0; qi < S->queue.size() && group.size() < kMaxBatchJobs;) {
                            Ticket& t = S->tickets[S->queue[qi]];
                            if (t.req.n > S->cfg.pack_max_records || recs + t.req.n > S->cfg.batch_records) {
                                ++qi;
                                continue;
                            }
                            group.push_back(&t);
                            const uint64_t need = L.ws + batch_bound(group, &S->cfg.params);
                            if (S->reserved() - L.ws + need + group_io + io_bytes(t.req) <= budget) {
                                charge = need;
                                group_io += io_bytes(t.req);
                                recs += t.req.n;
                                S->queue.erase(S->queue.begin() + (long)qi);
                            } else {
                                group.pop_back();
                                ++qi;
                            }
                        }
                    }
                    S->ws_charged += charge - L.ws;
                    L.ws = charge;
                    S->io_charged += group_io;
                    S->peak_reserved = std::max(S->peak_reserved, S->reserved());
                    break;
                }
                // nothing fits: an idle lane gives its workspace back first
                if (L.ws > 0 && !S->queue.empty()) {
                    ss_ctx* fresh = nullptr;
                    if (ss_create(S->device, L.stream, 0, &fresh) == SS_OK) {
                        (void)ss_destroy(L.ctx);
                        L.ctx = fresh;
                        S->ws_charged -= L.ws;
                        L.ws = 0;
                        S->cv.notify_all();  // other idle lanes look again (and give back too)
                        continue;
                    }
                }
                S->cv.wait(lk);
            }
        }
        const ss_status st = run_group(S, L, group);
        const double t_done = S->now();
        size_t held = 0;
        const bool have_held = ss_workspace_held(L.ctx, &held) == SS_OK;
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
            S->io_charged -= group_io;
            // from now on the lane is charged what its context really holds
            // (at most the charge it ran under)
            if (have_held && held < L.ws) {
                S->ws_charged -= L.ws - held;
                L.ws = held;
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
        if ((st = ss_create(device, L.stream, 0, &L.ctx)) != SS_OK) break;
        if (hipMalloc((void**)&L.d_m, kMaxBatchJobs * 8) != hipSuccess ||
            hipHostMalloc((void**)&L.h_m, kMaxBatchJobs * 8, hipHostMallocDefault) != hipSuccess) {
            st = SS_ENOMEM;
            break;
        }
    }
    if (st != SS_OK) {
        for (Lane& L : S->lanes) {
            if (L.ctx) ss_destroy(L.ctx);
            if (L.d_m) (void)hipFree(L.d_m);
            if (L.h_m) (void)hipHostFree(L.h_m);
            if (L.stream) (void)hipStreamDestroy(L.stream);
        }
        delete S;
        return st;
    }
    S->peak_reserved = S->reserved();
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
    if (!is_reduce(r->op) && r->val_bytes != 4 && r->val_bytes != 8) return SS_EINVAL;
    if (r->n >= (1ull << 31)) return SS_EINVAL;
    if (r->n && (!r->keys || !r->out_a || !r->out_b || (r->op != SS_OP_HISTOGRAM && !r->vals))) return SS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return SS_EINVAL;
    // a request that cannot fit even with every lane's workspace given back
    Ticket probe;
    probe.req = *r;
    if (r->n && batch_bound({&probe}, &S->cfg.params) + io_bytes(*r) > S->cfg.hbm_budget)
        return SS_ENOMEM;
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
        if (L.d_m) (void)hipFree(L.d_m);
        if (L.h_m) (void)hipHostFree(L.h_m);
        if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    delete S;
    return SS_OK;
}

}  // extern "C"
