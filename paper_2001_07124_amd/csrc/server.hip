// Continuous-batching request loop behind rhosvd_server_* (include/rhosvd.h).
//
// Requests (one decomposition each) queue in arrival order.  A scheduler
// thread admits them while a slot (a HIP stream of default priority) is free
// and their workspace fits in the caller's device pool (first-fit over free
// ranges), enqueues the whole decomposition on the slot's stream, and
// records an event.  As soon as a slot's event has completed, its pool range
// and the slot are released and the next waiting request can start, so new
// work joins while other requests are still running and their kernels
// overlap on the device.  The arithmetic of a request is exactly that of
// rhosvd_decompose on its own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rhosvd.h"

namespace {

double now_ms() {
    using clk = std::chrono::steady_clock;
    static const clk::time_point t0 = clk::now();
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

struct Request {
    // owned copies of the caller's descriptors
    std::vector<int64_t> dims;
    std::vector<int32_t> ranks;
    std::vector<void*> factors;
    rhosvd_tensor x{};
    rhosvd_params p{};
    rhosvd_output out{};
    size_t ws = 0, off = 0;
    int slot = -1;
    int state = RHOSVD_REQ_QUEUED;
    int32_t status = RHOSVD_OK;
    double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
};

// First-fit allocator over [0, size): free ranges by offset, 256-byte grain.
struct Pool {
    std::map<size_t, size_t> free;    // offset -> length
    explicit Pool(size_t size) { free[0] = size; }
    bool take(size_t n, size_t* off) {
        n = (n + 255) & ~static_cast<size_t>(255);
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, at = it->first + n;
                free.erase(it);
                if (rest) free[at] = rest;
                return true;
            }
        }
        return false;
    }
    void give(size_t off, size_t n) {
        n = (n + 255) & ~static_cast<size_t>(255);
        auto it = free.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free.erase(nx);
        }
        if (it != free.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free.erase(it);
            }
        }
    }
};

}  // namespace

struct rhosvd_server {
    rhosvd_ctx* ctx = nullptr;
    int device = 0;
    unsigned char* pool = nullptr;
    size_t pool_bytes = 0;
    Pool alloc{0};
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<int64_t> slot_req;         // ticket running in the slot, -1 if free
    std::deque<uint64_t> waiting;
    std::unordered_map<uint64_t, Request> reqs;
    uint64_t next = 1;
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    int lookahead = 8;                     // waiting requests scanned for one that fits
    uint64_t admitted = 0, completed = 0;

    void loop() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            bool progress = false;
            // completions
            for (size_t s = 0; s < streams.size(); ++s) {
                if (slot_req[s] < 0) continue;
                const hipError_t q = hipEventQuery(events[s]);
                if (q == hipErrorNotReady) continue;
                Request& r = reqs[static_cast<uint64_t>(slot_req[s])];
                r.t_done = now_ms();
                r.state = RHOSVD_REQ_DONE;
                if (q != hipSuccess) r.status = RHOSVD_EHIP;
                alloc.give(r.off, r.ws);
                slot_req[s] = -1;
                ++completed;
                progress = true;
            }
            // admissions: the oldest waiting requests that fit, while a slot is free
            for (size_t s = 0; s < streams.size(); ++s) {
                if (slot_req[s] >= 0 || waiting.empty()) continue;
                auto pick = waiting.end();
                size_t off = 0;
                const size_t scan = std::min<size_t>(waiting.size(), static_cast<size_t>(lookahead));
                for (size_t w = 0; w < scan; ++w) {
                    Request& r = reqs[waiting[w]];
                    if (alloc.take(r.ws, &off)) {
                        pick = waiting.begin() + static_cast<std::ptrdiff_t>(w);
                        break;
                    }
                }
                if (pick == waiting.end()) break;          // nothing fits until memory frees
                const uint64_t t = *pick;
                waiting.erase(pick);
                Request& r = reqs[t];
                r.off = off;
                r.slot = static_cast<int>(s);
                r.t_start = now_ms();
                r.state = RHOSVD_REQ_RUNNING;
                r.status = rhosvd_decompose(ctx, &r.x, &r.p, pool + off, r.ws, &r.out, streams[s]);
                if (r.status == RHOSVD_OK && hipEventRecord(events[s], streams[s]) != hipSuccess)
                    r.status = RHOSVD_EHIP;
                if (r.status != RHOSVD_OK) {
                    // nothing (more) runs for it: release at once
                    (void)hipStreamSynchronize(streams[s]);
                    alloc.give(r.off, r.ws);
                    r.state = RHOSVD_REQ_DONE;
                    r.t_done = now_ms();
                    ++completed;
                } else {
                    slot_req[s] = static_cast<int64_t>(t);
                }
                ++admitted;
                progress = true;
            }
            cv.notify_all();
            bool busy = !waiting.empty();
            for (int64_t q : slot_req) busy = busy || q >= 0;
            if (stop && !busy) break;
            if (!progress) {
                if (busy)
                    cv.wait_for(lk, std::chrono::microseconds(20));
                else
                    cv.wait(lk, [&] { return stop || !waiting.empty(); });
            }
        }
    }
};

extern "C" {

int32_t rhosvd_server_create(rhosvd_ctx* ctx, int32_t device, void* pool, size_t pool_bytes,
                             int32_t max_slots, rhosvd_server** out) {
    if (!ctx || !pool || !out || pool_bytes < 4096 || max_slots < 1 || max_slots > 64)
        return RHOSVD_EINVAL;
    if (reinterpret_cast<uintptr_t>(pool) % 256 != 0) return RHOSVD_EINVAL;
    *out = nullptr;
    rhosvd_server* S = new (std::nothrow) rhosvd_server;
    if (!S) return RHOSVD_ENOMEM;
    S->ctx = ctx;
    S->device = device;
    S->pool = static_cast<unsigned char*>(pool);
    S->pool_bytes = pool_bytes & ~static_cast<size_t>(255);
    S->alloc = Pool(S->pool_bytes);
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
    for (int s = 0; s < max_slots; ++s) {
        hipStream_t st;
        hipEvent_t ev;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) break;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamDestroy(st);
            break;
        }
        S->streams.push_back(st);
        S->events.push_back(ev);
        S->slot_req.push_back(-1);
    }
    if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
    if (static_cast<int>(S->streams.size()) != max_slots) {
        for (auto st : S->streams) (void)hipStreamDestroy(st);
        for (auto ev : S->events) (void)hipEventDestroy(ev);
        delete S;
        return RHOSVD_EHIP;
    }
    S->worker = std::thread([S] { S->loop(); });
    *out = S;
    return RHOSVD_OK;
}

int32_t rhosvd_server_submit(rhosvd_server* S, const rhosvd_tensor* x, const rhosvd_params* p,
                             const rhosvd_output* out, uint64_t* ticket) {
    if (!S || !x || !p || !out || !ticket || !x->dims || !p->ranks || !out->factors)
        return RHOSVD_EINVAL;
    if (x->order < 2 || x->order > RHOSVD_MAX_ORDER) return RHOSVD_EINVAL;
    size_t ws = 0;
    const int32_t rc = rhosvd_workspace_size(x, p, &ws);
    if (rc != RHOSVD_OK) return rc;
    if (!x->data || !out->core) return RHOSVD_EINVAL;
    for (int n = 0; n < x->order; ++n)
        if (!out->factors[n]) return RHOSVD_EINVAL;
    if (p->mode_order) return RHOSVD_EUNSUPPORTED;
    if (((ws + 255) & ~static_cast<size_t>(255)) > S->pool_bytes) return RHOSVD_ENOMEM;
    Request r;
    const int N = x->order;
    r.dims.assign(x->dims, x->dims + N);
    r.ranks.assign(p->ranks, p->ranks + N);
    r.factors.assign(out->factors, out->factors + N);
    r.x = *x;
    r.x.dims = r.dims.data();
    r.p = *p;
    r.p.ranks = r.ranks.data();
    r.p.mode_order = nullptr;
    r.out = *out;
    r.ws = ws;
    r.t_submit = now_ms();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        const uint64_t t = S->next++;
        auto& slot = S->reqs[t];
        slot = std::move(r);
        // the vectors moved: re-point the descriptors at the owned copies
        slot.x.dims = slot.dims.data();
        slot.p.ranks = slot.ranks.data();
        slot.out.factors = slot.factors.data();
        S->waiting.push_back(t);
        *ticket = t;
    }
    S->cv.notify_all();
    return RHOSVD_OK;
}

int32_t rhosvd_server_poll(rhosvd_server* S, uint64_t ticket, int32_t* state, double* times_ms) {
    if (!S || !state) return RHOSVD_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return RHOSVD_EINVAL;
    const Request& r = it->second;
    *state = r.state;
    if (times_ms) {
        times_ms[0] = r.t_submit;
        times_ms[1] = r.t_start;
        times_ms[2] = r.t_done;
    }
    return r.state == RHOSVD_REQ_DONE ? r.status : RHOSVD_OK;
}

int32_t rhosvd_server_release(rhosvd_server* S, uint64_t ticket) {
    if (!S) return RHOSVD_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end() || it->second.state != RHOSVD_REQ_DONE) return RHOSVD_EINVAL;
    S->reqs.erase(it);
    return RHOSVD_OK;
}

int32_t rhosvd_server_drain(rhosvd_server* S) {
    if (!S) return RHOSVD_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv.wait(lk, [&] {
        if (!S->waiting.empty()) return false;
        for (int64_t q : S->slot_req)
            if (q >= 0) return false;
        return true;
    });
    return RHOSVD_OK;
}

void rhosvd_server_destroy(rhosvd_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (auto st : S->streams) (void)hipStreamDestroy(st);
    for (auto ev : S->events) (void)hipEventDestroy(ev);
    delete S;
}

}  // extern "C"
