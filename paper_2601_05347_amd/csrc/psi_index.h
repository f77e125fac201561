// Host-side state of an index and the helpers shared by the C ABI files.
#pragma once
#include <hip/hip_runtime.h>

#include <deque>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/psi.h"
#include "psi_kern.h"

namespace psi {

// Grow-only device buffer. ensure() may drop the contents; grow_keep()
// preserves them (stream-ordered copy).
struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
    ~Buf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    psi_status ensure(size_t need) {
        if (need <= bytes) return PSI_OK;
        release();
        size_t want = need + need / 4 + 256;
        if (hipMalloc(&p, want) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            if (hipMalloc(&p, need) != hipSuccess) {
                p = nullptr;
                (void)hipGetLastError();
                return PSI_E_NOMEM;
            }
            want = need;
        }
        bytes = want;
        return PSI_OK;
    }
    psi_status grow_keep(size_t need, size_t keep, hipStream_t st) {
        if (need <= bytes) return PSI_OK;
        void* q = nullptr;
        size_t want = need + need / 2 + 256;
        if (hipMalloc(&q, want) != hipSuccess) {
            (void)hipGetLastError();
            want = need;
            if (hipMalloc(&q, want) != hipSuccess) {
                (void)hipGetLastError();
                return PSI_E_NOMEM;
            }
        }
        if (p && keep) {
            if (hipMemcpyAsync(q, p, keep, hipMemcpyDeviceToDevice, st) != hipSuccess) return PSI_E_HIP;
            if (hipStreamSynchronize(st) != hipSuccess) return PSI_E_HIP;
        }
        release();
        p = q;
        bytes = want;
        return PSI_OK;
    }
    // Stream-ordered variants for the index's hot paths: the new block is
    // allocated at once (twice the size asked for, so that a stream of
    // growing updates reallocates rarely), the old one (its contents copied
    // on `st` first by grow_keep_q) goes to `grave` and is freed once the
    // stream is idle, so neither call waits for queued work. need <= bytes
    // does nothing.
    psi_status ensure_q(size_t need, std::vector<void*>& grave) {
        if (need <= bytes) return PSI_OK;
        void* q = nullptr;
        size_t want = 2 * need + 256;
        if (hipMalloc(&q, want) != hipSuccess) {
            (void)hipGetLastError();
            want = need;
            if (hipMalloc(&q, want) != hipSuccess) {
                (void)hipGetLastError();
                return PSI_E_NOMEM;
            }
        }
        if (p) grave.push_back(p);
        p = q;
        bytes = want;
        return PSI_OK;
    }
    psi_status grow_keep_q(size_t need, hipStream_t st, std::vector<void*>& grave) {
        if (need <= bytes) return PSI_OK;
        void* q = nullptr;
        size_t want = 2 * need + 256;
        if (hipMalloc(&q, want) != hipSuccess) {
            (void)hipGetLastError();
            want = need;
            if (hipMalloc(&q, want) != hipSuccess) {
                (void)hipGetLastError();
                return PSI_E_NOMEM;
            }
        }
        if (p) {
            if (hipMemcpyAsync(q, p, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) {
                (void)hipGetLastError();
                (void)hipFree(q);
                return PSI_E_HIP;
            }
            grave.push_back(p);
        }
        p = q;
        bytes = want;
        return PSI_OK;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Upper bounds of the device state's sizes, as the host tracks them.
struct Bounds {
    uint64_t L = 0, slot_top = 0, n_free = 0, n_live = 0, next_id = 0;
};
// An update whose commit the host has not seen yet: its event, the pinned
// slot its DevTree head is copied to, and how much it may have grown the
// state. `stale`: a later build replaced the state it describes.
struct Inflight {
    hipEvent_t ev = nullptr;
    uint32_t slot = 0;
    Bounds delta;
    bool stale = false;
};
constexpr uint32_t MIRROR_SLOTS = 64;  // updates in flight before a call waits

// Per-family kernel timing with HIP events (enabled on demand).
struct ProfFamily {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    double ms = 0.0;
    uint64_t launches = 0;
    uint64_t bytes = 0;
};
struct Prof {
    bool on = false;
    std::string only;  // when not empty: the one family bracketed
    std::map<std::string, ProfFamily> fam;
    std::vector<hipEvent_t> pool;
    hipEvent_t take() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        // timing only: no system-scope fence (no cache writeback between the
        // kernels the events bracket)
        hipEvent_t e = nullptr;
        (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
        return e;
    }
    void resolve() {
        for (auto& kv : fam) {
            for (auto& pr : kv.second.pending) {
                float ms = 0.f;
                if (hipEventSynchronize(pr.second) == hipSuccess &&
                    hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess)
                    kv.second.ms += ms;
                pool.push_back(pr.first);
                pool.push_back(pr.second);
            }
            kv.second.pending.clear();
        }
    }
    ~Prof() {
        for (auto& kv : fam)
            for (auto& pr : kv.second.pending) {
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

// Radix-sort workspace: histograms, digit offsets, look-back status words and
// the two ping-pong pair buffers.
struct Sorter {
    Buf hist, off, ctr, status, k[2], i[2];
    Buf bk, bseg, shist, soff;  // two-level build sort: bucket tables, big-bucket segments
    Buf kmax;                   // largest key of a build (u64)
    Buf xt;                     // chunked bucket passes: counts, digit offsets, chunk tables
    uint32_t epoch = 0;
    uint64_t status_words = 0;
};

struct Scratch {
    Buf a, b, c, d, e, f, g, h2, s;  // general purpose, sized per call
};

}  // namespace psi

struct psi_index_s {
    int D = 2;
    int curve = 0;
    uint32_t phi = 32;
    uint32_t C = 64;  // slot stride (2 phi rounded up to a multiple of 4)
    uint32_t B = 8;
    uint32_t flags = 0;
    hipStream_t st = nullptr;

    // The sizes of the tree (leaf count, live points, next id, slot and
    // free-stack tops, current directory buffer, node layout) live on the
    // device in `dev` (a DevTree) and change only in stream order. The host
    // keeps `base`, their exact values as of the last update it has seen
    // complete (or the last wait), plus per-update growth bounds of the
    // updates still in flight; buffers and grids are sized by base + those
    // bounds, so no call needs the device's answer before it returns.
    psi::Buf dev;
    psi::Bounds base;
    std::deque<psi::Inflight> inflight;
    psi::DevTree* mirror = nullptr;  // pinned [MIRROR_SLOTS] DevTree heads
    uint32_t mirror_next = 0;
    std::vector<hipEvent_t> ev_pool;
    bool unknown = false;   // a replayed graph changed the state: wait before sizing
    uint64_t gen = 1;       // bumped by every change that stales a captured graph
    std::vector<void*> grave;  // replaced device blocks, freed once the stream is idle

    // id -> key table (DEAD_KEY for deleted or never used ids)
    psi::Buf idkey;

    // leaf storage: slot s holds [D][C] coordinates then [C] ids (u32)
    psi::Buf slots;
    psi::Buf free_stack;    // freed slots, reused before bumping

    // leaf directory (double-buffered for updates): records and pivots
    psi::Buf leaf[2], pkey[2], pid[2];

    // node levels 0..h-1, level-major from the root
    psi::Buf inner;
    psi::Buf cinner, cleaf;  // packed boxes of the inner nodes and of the leaves
    psi::Buf psample;        // every PSAMPLE-th pivot (routing's first steps)
    bool boxes_fresh = false;  // packed boxes match the current tree
    uint64_t L_cap = 0;        // leaves the node buffers and packed boxes are sized for

    uint32_t bucket_top = ~0u;  // bucket bits of the last two-level build sort

    psi::Buf err;      // device u32 error bits
    void* pinned = nullptr;  // host readback area (4 KiB)
    psi::Sorter sorter;    // builds and updates
    psi::Sorter qsorter;   // query ordering: queries may run beside an update
    psi::Buf qkeys;        // curve keys of a query batch
    psi::Scratch scr;
    hipStream_t aux_st = nullptr;  // a second stream the index's queries run on (a server's)
    psi::Prof prof;
    psi::Buf qstats;           // kNN walk counts (psi_query_stats)
    psi::KnnTuning knn_tune;   // psi_set_tuning
    uint32_t order_bits = 24;  // top key bits the query order sorts on
    bool qstats_on = false;

    uint64_t slot_words() const { return (uint64_t)(D + 1) * C; }
    psi::DevTree* dt() const { return dev.as<psi::DevTree>(); }
    // View for query kernels: sizes and the directory come from dt at launch.
    psi::TreeView view() const;
};

namespace psi {

// Records launches of one kernel family between HIP events when profiling.
struct ProfScope {
    psi_index ix;
    const char* fam;
    uint64_t bytes;
    hipEvent_t a = nullptr;
    bool on;
    ProfScope(psi_index x, const char* f, uint64_t b)
        : ix(x), fam(f), bytes(b), on(x->prof.on && (x->prof.only.empty() || x->prof.only == f)) {
        if (on) {
            a = ix->prof.take();
            (void)hipEventRecord(a, ix->st);
        }
    }
    ~ProfScope() {
        if (on) {
            hipEvent_t e = ix->prof.take();
            (void)hipEventRecord(e, ix->st);
            ProfFamily& f = ix->prof.fam[fam];
            f.pending.push_back({a, e});
            f.launches += 1;
            f.bytes += bytes;
        }
    }
};

psi_status hip_ok(hipError_t e);
// True while `st` is being captured into a graph: no allocation, no waiting.
bool capturing(hipStream_t st);
// Buf::ensure for paths that may run under graph capture: growing a buffer
// there is refused (PSI_E_STATE); a call outside capture sizes it first.
// Growth never waits (the old block is freed once the stream is idle) and
// stales captured graphs.
psi_status ensure_q(psi_index ix, Buf& b, size_t need);
psi_status grow_keep_q(psi_index ix, Buf& b, size_t need);

// Host view of the device state (psi_api.hip).
// Retires the updates that have completed (non-blocking) and frees replaced
// blocks once the stream is idle.
void poll(psi_index ix);
// Upper bounds of the state once every queued update has run (waits only if
// a replayed graph left the state unknown).
psi_status bounds(psi_index ix, Bounds* out);
// Waits for the stream and makes `base` exact (no update left in flight).
psi_status settle(psi_index ix);
// After an update's kernels: mirror the DevTree head to pinned memory behind
// an event, so a later call can take exact sizes without waiting.
psi_status track_update(psi_index ix, const Bounds& delta);
// Sizes the node buffers and packed boxes for up to L leaves, launches the
// node levels of the layout in dt (at most the height of L leaves).
psi_status build_nodes(psi_index ix, uint64_t L_bound);
// Exact tree view for exports (after settle()): leaf count, height and the
// current directory from the state.
psi::TreeView exact_view(psi_index ix, std::vector<psi::LevelInfo>* lv = nullptr);
// sorter: the workspace (null: the index's update workspace).
psi_status sort_pairs(psi_index ix, const uint64_t* kin, const uint32_t* iin, uint32_t id_base, uint64_t n,
                      bool id_digits, bool hist_ready, int* which, const char* fam, uint32_t key_shift0 = 0,
                      int key_passes = 8, Sorter* sorter = nullptr);
psi_status readback(psi_index ix, const void* dev, size_t bytes);  // into ix->pinned, waits

// updates (psi_update.hip)
// before_apply (may be null): the stream waits for this event before the
// first kernel that changes what queries read (leaves, directory, nodes);
// the batch's encode, sort, routing and planning run before that.
psi_status do_insert(psi_index ix, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids,
                     hipEvent_t before_apply = nullptr);
psi_status do_delete(psi_index ix, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted,
                     hipEvent_t before_apply = nullptr);
psi_status do_build(psi_index ix, const uint32_t* d_pts, uint64_t n);
// Curve keys of n points into keys[0 .. n) and the pairs (key, id_base + i)
// sorted by (key, id) into sorter.k/i[*which]; requires n > 0.
psi_status encode_sort(psi_index ix, const uint32_t* d_pts, uint64_t n, uint64_t* keys, uint32_t id_base,
                       int* which);
// Both directory buffers sized for `leaves` leaves (contents kept).
psi_status ensure_dirs(psi_index ix, uint64_t leaves);
// The directory buffers as kernel arguments take them.
psi::Dirs dirs_of(psi_index ix);
// Processing order of a query batch (curve keys of the points or box centres
// in qkeys, input order; *order null or the positions sorted by key); latches
// ERR_RANGE for out-of-range query points.
psi_status query_order(psi_index ix, const uint32_t* d_items, uint64_t n, bool boxes, const uint32_t** order);

}  // namespace psi
