// Serving a resident index: continuous batching of mixed requests with
// device overlap.
//
// Requests (insert, delete, kNN, range count, range report) take effect in
// submission order: each sees exactly the updates submitted before it, as if
// they ran one at a time. The server groups the queue into epochs -- maximal
// runs of updates or of queries -- admitted while their estimated device
// footprint fits a budget:
//  * an update epoch runs on the update stream. Consecutive inserts become
//    one batch (ids are handed out in submission order, so merging changes
//    no id). An update's first part (encode, sort, routing, planning) reads
//    only the current directory and writes its own workspace, so it runs
//    while the queries of the previous epoch still read the tree; the
//    update waits for those queries only before its first write to the
//    leaves, the directory or the nodes;
//  * a query epoch runs on the query stream after the last update epoch has
//    completed. kNN requests with the same k share one launch; every query
//    uses the index's query workspace, separate from the update's;
//  * no call waits for the device except when the budget is full (the
//    oldest epoch is waited for) or the caller asks (psi_server_wait).
// Completion times are HIP events, reported in ms since the server was
// created.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <new>
#include <vector>

#include "psi_index.h"

using namespace psi;

namespace psi {
namespace {

// u64 exclusive scan of n counts into off[0..n] (one workgroup; a request's
// boxes number at most a few tens of thousands) and the same offsets clamped
// to cap (the report writes into the caller's buffer of cap ids).
__global__ __launch_bounds__(1024) void k_offsets_u64(const uint64_t* __restrict__ cnt, uint64_t n,
                                                      uint64_t* __restrict__ off, uint64_t* __restrict__ clamped,
                                                      uint64_t cap) {
    __shared__ uint64_t s_part[1024];
    __shared__ uint64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint64_t b = 0; b < n; b += 1024) {
        const uint64_t i = b + threadIdx.x;
        const uint64_t v = i < n ? cnt[i] : 0;
        s_part[threadIdx.x] = v;
        __syncthreads();
        for (uint32_t o = 1; o < 1024; o <<= 1) {
            const uint64_t t = threadIdx.x >= o ? s_part[threadIdx.x - o] : 0;
            __syncthreads();
            s_part[threadIdx.x] += t;
            __syncthreads();
        }
        const uint64_t excl = s_carry + s_part[threadIdx.x] - v;
        if (i < n) {
            off[i] = excl;
            clamped[i] = excl < cap ? excl : cap;
        }
        __syncthreads();
        if (threadIdx.x == 1023) s_carry += s_part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        off[n] = s_carry;
        clamped[n] = s_carry < cap ? s_carry : cap;
    }
}

// Grow-only device buffer whose replaced blocks wait for the server to idle.
struct SBuf {
    void* p = nullptr;
    size_t bytes = 0;
    psi_status need(size_t n, std::vector<void*>& grave) {
        if (n <= bytes) return PSI_OK;
        void* q = nullptr;
        const size_t want = n + n / 2 + 256;
        if (hipMalloc(&q, want) != hipSuccess) {
            (void)hipGetLastError();
            return PSI_E_NOMEM;
        }
        if (p) grave.push_back(p);
        p = q;
        bytes = want;
        return PSI_OK;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

enum : uint32_t { QUEUED = 0, DISPATCHED = 1, DONE = 2 };

struct Ticket {
    psi_request req;
    uint64_t fp = 0;        // estimated device bytes while in flight
    uint32_t state = QUEUED;
    psi_status status = PSI_OK;
    int64_t epoch = -1;     // index into epochs once dispatched
};

struct Epoch {
    hipEvent_t done = nullptr;
    bool complete = false;
    double ms = 0;
    uint64_t fp = 0;
};

bool is_update(uint32_t kind) { return kind == PSI_REQ_INSERT || kind == PSI_REQ_DELETE; }

}  // namespace
}  // namespace psi

struct psi_server_s {
    psi_index ix = nullptr;
    hipStream_t home = nullptr;  // the index's stream before the server took it
    hipStream_t su = nullptr, sq = nullptr;
    uint64_t budget = 0, in_flight = 0;
    hipEvent_t base = nullptr;
    hipEvent_t last_upd = nullptr, last_qry = nullptr;  // latest epochs of each kind (not owned)
    std::vector<Ticket> tickets;
    std::deque<uint64_t> queue;          // submitted, not dispatched (ticket numbers)
    std::vector<Epoch> epochs;
    size_t first_open = 0;               // epochs before this one are complete
    std::vector<void*> grave;
    SBuf ins_pts, ins_ids, kq, kids, kd2, rcnt, rclamp;
};

namespace psi {
namespace {

uint64_t footprint(const psi_request& r, int D) {
    switch (r.kind) {
        case PSI_REQ_INSERT: return r.n * (4ull * D + 64);
        case PSI_REQ_DELETE: return r.n * 64;
        case PSI_REQ_KNN: return r.n * (4ull * D + 12ull * r.k + 32);
        case PSI_REQ_RANGE_COUNT: return r.n * (8ull * D + 16);
        default: return r.n * (8ull * D + 32) + r.ids_cap * 4;
    }
}

// Retires completed epochs (non-blocking unless `block_oldest`).
void retire(psi_server s, bool block_oldest) {
    while (s->first_open < s->epochs.size()) {
        Epoch& e = s->epochs[s->first_open];
        if (block_oldest) {
            (void)hipEventSynchronize(e.done);
            block_oldest = false;
        }
        const hipError_t q = hipEventQuery(e.done);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) (void)hipGetLastError();
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, s->base, e.done) != hipSuccess) (void)hipGetLastError();
        e.ms = ms;
        e.complete = true;
        s->in_flight -= std::min(s->in_flight, e.fp);
        ++s->first_open;
    }
    if (s->first_open == s->epochs.size() && !s->grave.empty() && hipStreamQuery(s->su) == hipSuccess &&
        hipStreamQuery(s->sq) == hipSuccess) {
        for (void* p : s->grave) (void)hipFree(p);
        s->grave.clear();
    }
}

psi_status wait_ready(hipStream_t st, const psi_request& r) {
    if (!r.ready_event) return PSI_OK;
    return hip_ok(hipStreamWaitEvent(st, static_cast<hipEvent_t>(r.ready_event), 0));
}

psi_status run_updates(psi_server s, const std::vector<uint64_t>& run) {
    psi_index ix = s->ix;
    hipStream_t st = s->su;
    psi_status st_ok = PSI_OK;
    hipEvent_t before = s->last_qry;  // the first change to the tree waits for the queries before it
    size_t i = 0;
    while (i < run.size()) {
        Ticket& t = s->tickets[run[i]];
        if (t.req.kind == PSI_REQ_INSERT) {
            size_t j = i;
            uint64_t M = 0;
            while (j < run.size() && s->tickets[run[j]].req.kind == PSI_REQ_INSERT) M += s->tickets[run[j++]].req.n;
            psi_status r;
            for (size_t x = i; x < j; ++x)
                if ((r = wait_ready(st, s->tickets[run[x]].req)) != PSI_OK) return r;
            if (M == 0) {  // nothing to insert
                i = j;
                continue;
            }
            if (j - i == 1) {
                r = do_insert(ix, t.req.d_in, t.req.n, t.req.d_ids, before);
            } else {
                // one batch: the payloads side by side, the new ids copied back
                const uint64_t row = 4ull * ix->D;
                if ((r = s->ins_pts.need(M * row, s->grave)) != PSI_OK) return r;
                if ((r = s->ins_ids.need(M * 4, s->grave)) != PSI_OK) return r;
                uint64_t o = 0;
                for (size_t x = i; x < j; ++x) {
                    const psi_request& q = s->tickets[run[x]].req;
                    if ((r = hip_ok(hipMemcpyAsync(s->ins_pts.as<char>() + o * row, q.d_in, q.n * row,
                                                   hipMemcpyDeviceToDevice, st))) != PSI_OK)
                        return r;
                    o += q.n;
                }
                r = do_insert(ix, s->ins_pts.as<uint32_t>(), M, s->ins_ids.as<uint32_t>(), before);
                o = 0;
                for (size_t x = i; x < j && r == PSI_OK; ++x) {
                    const psi_request& q = s->tickets[run[x]].req;
                    if (q.d_ids)
                        r = hip_ok(hipMemcpyAsync(q.d_ids, s->ins_ids.as<uint32_t>() + o, q.n * 4,
                                                  hipMemcpyDeviceToDevice, st));
                    o += q.n;
                }
            }
            if (r != PSI_OK) return r;
            before = nullptr;
            i = j;
        } else {
            psi_status r = wait_ready(st, t.req);
            if (r == PSI_OK) r = do_delete(ix, t.req.d_in, t.req.n, t.req.d_out, before);
            if (r != PSI_OK) return r;
            before = nullptr;
            ++i;
        }
    }
    return st_ok;
}

psi_status run_queries(psi_server s, const std::vector<uint64_t>& run) {
    psi_index ix = s->ix;
    hipStream_t st = s->sq;
    psi_status r;
    if (s->last_upd && (r = hip_ok(hipStreamWaitEvent(st, s->last_upd, 0))) != PSI_OK) return r;
    for (uint64_t tn : run)
        if ((r = wait_ready(st, s->tickets[tn].req)) != PSI_OK) return r;
    const int D = ix->D;
    // kNN: one launch per k
    std::vector<uint32_t> ks;
    for (uint64_t tn : run)
        if (s->tickets[tn].req.kind == PSI_REQ_KNN) ks.push_back(s->tickets[tn].req.k);
    std::sort(ks.begin(), ks.end());
    ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
    for (uint32_t k : ks) {
        std::vector<const psi_request*> g;
        uint64_t nq = 0;
        for (uint64_t tn : run) {
            const psi_request& q = s->tickets[tn].req;
            if (q.kind == PSI_REQ_KNN && q.k == k) {
                g.push_back(&q);
                nq += q.n;
            }
        }
        if (g.size() == 1) {
            if ((r = psi_knn(ix, g[0]->d_in, g[0]->n, k, g[0]->d_ids, g[0]->d_out)) != PSI_OK) return r;
            continue;
        }
        const uint64_t row = 4ull * D;
        if ((r = s->kq.need(nq * row, s->grave)) != PSI_OK) return r;
        if ((r = s->kids.need(nq * k * 4, s->grave)) != PSI_OK) return r;
        if ((r = s->kd2.need(nq * k * 8, s->grave)) != PSI_OK) return r;
        uint64_t o = 0;
        for (const psi_request* q : g) {
            if ((r = hip_ok(hipMemcpyAsync(s->kq.as<char>() + o * row, q->d_in, q->n * row, hipMemcpyDeviceToDevice,
                                           st))) != PSI_OK)
                return r;
            o += q->n;
        }
        if ((r = psi_knn(ix, s->kq.as<uint32_t>(), nq, k, s->kids.as<uint32_t>(), s->kd2.as<uint64_t>())) != PSI_OK)
            return r;
        o = 0;
        for (const psi_request* q : g) {
            if ((r = hip_ok(hipMemcpyAsync(q->d_ids, s->kids.as<uint32_t>() + o * k, q->n * k * 4,
                                           hipMemcpyDeviceToDevice, st))) != PSI_OK)
                return r;
            if ((r = hip_ok(hipMemcpyAsync(q->d_out, s->kd2.as<uint64_t>() + o * k, q->n * k * 8,
                                           hipMemcpyDeviceToDevice, st))) != PSI_OK)
                return r;
            o += q->n;
        }
    }
    // ranges: one request at a time (count, offsets, report)
    for (uint64_t tn : run) {
        const psi_request& q = s->tickets[tn].req;
        if (q.kind == PSI_REQ_RANGE_COUNT) {
            if ((r = psi_range_count(ix, q.d_in, q.n, q.d_out)) != PSI_OK) return r;
        } else if (q.kind == PSI_REQ_RANGE_REPORT) {
            if ((r = s->rcnt.need(q.n * 8 + 8, s->grave)) != PSI_OK) return r;
            if ((r = s->rclamp.need(q.n * 8 + 8, s->grave)) != PSI_OK) return r;
            if ((r = psi_range_count(ix, q.d_in, q.n, s->rcnt.as<uint64_t>())) != PSI_OK) return r;
            hipLaunchKernelGGL(k_offsets_u64, dim3(1), dim3(1024), 0, st, s->rcnt.as<uint64_t>(), q.n, q.d_out,
                               s->rclamp.as<uint64_t>(), q.ids_cap);
            if ((r = hip_ok(hipGetLastError())) != PSI_OK) return r;
            if (q.ids_cap > 0 && (r = psi_range_report(ix, q.d_in, q.n, s->rclamp.as<uint64_t>(), q.d_ids)) != PSI_OK)
                return r;
        }
    }
    return PSI_OK;
}

// Dispatches queued requests as epochs, admitting by budget.
psi_status progress(psi_server s) {
    retire(s, false);
    while (!s->queue.empty()) {
        const bool upd = is_update(s->tickets[s->queue.front()].req.kind);
        std::vector<uint64_t> run;
        uint64_t fp = 0;
        while (!s->queue.empty() && is_update(s->tickets[s->queue.front()].req.kind) == upd) {
            Ticket& t = s->tickets[s->queue.front()];
            if (t.fp > s->budget) {  // can never fit: refused, in order
                if (!run.empty()) break;
                t.state = DONE;
                t.status = PSI_E_CAPACITY;
                s->queue.pop_front();
                continue;
            }
            if (s->in_flight + fp + t.fp > s->budget) {
                if (!run.empty()) break;  // dispatch what fits first
                if (s->first_open == s->epochs.size()) break;  // nothing to wait for (cannot happen)
                retire(s, true);  // wait for the oldest epoch to free its share
                continue;
            }
            fp += t.fp;
            run.push_back(s->queue.front());
            s->queue.pop_front();
        }
        if (run.empty()) continue;
        psi_index ix = s->ix;
        psi_status r;
        Epoch e;
        e.fp = fp;
        if ((r = hip_ok(hipEventCreate(&e.done))) != PSI_OK) return r;
        if (upd) {
            ix->st = s->su;
            r = run_updates(s, run);
            if (r == PSI_OK) r = hip_ok(hipEventRecord(e.done, s->su));
        } else {
            ix->st = s->sq;  // queries are issued on the query stream
            r = run_queries(s, run);
            ix->st = s->su;
            if (r == PSI_OK) r = hip_ok(hipEventRecord(e.done, s->sq));
        }
        const int64_t eid = (int64_t)s->epochs.size();
        s->epochs.push_back(e);
        if (upd) s->last_upd = e.done;
        else s->last_qry = e.done;
        s->in_flight += fp;
        for (uint64_t tn : run) {
            s->tickets[tn].state = DISPATCHED;
            s->tickets[tn].epoch = eid;
            if (r != PSI_OK) s->tickets[tn].status = r;
        }
        if (r != PSI_OK) return r;
    }
    return PSI_OK;
}

}  // namespace
}  // namespace psi

extern "C" {

psi_status psi_server_create(psi_index ix, uint64_t budget_bytes, psi_server* out) {
    if (!ix || !out || budget_bytes == 0) return PSI_E_ARG;
    *out = nullptr;
    psi_status s = settle(ix);
    if (s != PSI_OK) return s;
    psi_server sv = new (std::nothrow) psi_server_s;
    if (!sv) return PSI_E_NOMEM;
    sv->ix = ix;
    sv->home = ix->st;
    sv->budget = budget_bytes;
    s = hip_ok(hipStreamCreateWithFlags(&sv->su, hipStreamNonBlocking));
    if (s == PSI_OK) s = hip_ok(hipStreamCreateWithFlags(&sv->sq, hipStreamNonBlocking));
    if (s == PSI_OK) s = hip_ok(hipEventCreate(&sv->base));
    if (s == PSI_OK) s = hip_ok(hipEventRecord(sv->base, sv->su));
    if (s == PSI_OK) s = hip_ok(hipEventSynchronize(sv->base));
    if (s != PSI_OK) {
        if (sv->su) (void)hipStreamDestroy(sv->su);
        if (sv->sq) (void)hipStreamDestroy(sv->sq);
        if (sv->base) (void)hipEventDestroy(sv->base);
        delete sv;
        return s;
    }
    ix->st = sv->su;
    ix->aux_st = sv->sq;
    *out = sv;
    return PSI_OK;
}

psi_status psi_server_destroy(psi_server sv) {
    if (!sv) return PSI_E_ARG;
    psi_status s = progress(sv);
    (void)hipStreamSynchronize(sv->su);
    (void)hipStreamSynchronize(sv->sq);
    for (Epoch& e : sv->epochs) (void)hipEventDestroy(e.done);
    for (void* p : sv->grave) (void)hipFree(p);
    for (SBuf* b : {&sv->ins_pts, &sv->ins_ids, &sv->kq, &sv->kids, &sv->kd2, &sv->rcnt, &sv->rclamp})
        if (b->p) (void)hipFree(b->p);
    sv->ix->st = sv->home;
    sv->ix->aux_st = nullptr;
    (void)hipStreamDestroy(sv->su);
    (void)hipStreamDestroy(sv->sq);
    (void)hipEventDestroy(sv->base);
    delete sv;
    return s;
}

psi_status psi_server_submit(psi_server sv, const psi_request* req, uint64_t* h_ticket) {
    if (!sv || !req || !h_ticket) return PSI_E_ARG;
    const psi_request& r = *req;
    const bool need_in = r.n > 0;
    switch (r.kind) {
        case PSI_REQ_INSERT:
        case PSI_REQ_DELETE: break;
        case PSI_REQ_KNN:
            if (r.k == 0 || r.k > 128 || (need_in && (!r.d_ids || !r.d_out))) return PSI_E_ARG;
            break;
        case PSI_REQ_RANGE_COUNT:
            if (need_in && !r.d_out) return PSI_E_ARG;
            break;
        case PSI_REQ_RANGE_REPORT:
            if (!r.d_out || (r.ids_cap && !r.d_ids)) return PSI_E_ARG;
            break;
        default: return PSI_E_ARG;
    }
    if (need_in && !r.d_in) return PSI_E_ARG;
    Ticket t;
    t.req = r;
    t.fp = footprint(r, sv->ix->D);
    *h_ticket = sv->tickets.size();
    sv->tickets.push_back(t);
    sv->queue.push_back(*h_ticket);
    return PSI_OK;
}

psi_status psi_server_poll(psi_server sv, uint64_t ticket, int* h_done, double* h_done_ms) {
    if (!sv || !h_done || ticket >= sv->tickets.size()) return PSI_E_ARG;
    psi_status s = progress(sv);
    retire(sv, false);
    const Ticket& t = sv->tickets[ticket];
    *h_done = 0;
    if (t.state == DONE) {
        *h_done = 1;
        return t.status;
    }
    if (t.state == DISPATCHED && sv->epochs[t.epoch].complete) {
        *h_done = 1;
        if (h_done_ms) *h_done_ms = sv->epochs[t.epoch].ms;
        return t.status != PSI_OK ? t.status : s;
    }
    return s;
}

psi_status psi_server_wait(psi_server sv, uint64_t ticket, double* h_done_ms) {
    if (!sv || ticket >= sv->tickets.size()) return PSI_E_ARG;
    psi_status s = progress(sv);
    if (s != PSI_OK) return s;
    const Ticket& t = sv->tickets[ticket];
    if (t.state == DISPATCHED) {
        while (!sv->epochs[t.epoch].complete) retire(sv, true);
        if (h_done_ms) *h_done_ms = sv->epochs[t.epoch].ms;
    }
    return t.status;
}

psi_status psi_server_flush(psi_server sv) {
    if (!sv) return PSI_E_ARG;
    return progress(sv);
}

}  // extern "C"
