// Host-side state of an index and the helpers shared by the C ABI files.
#pragma once
#include <hip/hip_runtime.h>

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
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Per-family kernel timing with HIP events (enabled on demand).
struct ProfFamily {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    double ms = 0.0;
    uint64_t launches = 0;
    uint64_t bytes = 0;
};
struct Prof {
    bool on = false;
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
    uint32_t C = 64;  // slot capacity (2 phi rounded up to a multiple of 4)
    uint32_t B = 8;
    uint32_t flags = 0;
    hipStream_t st = nullptr;

    // id -> key table (DEAD_KEY for deleted or never used ids)
    psi::Buf idkey;
    uint32_t next_id = 0;
    uint64_t n_live = 0;

    // leaf storage: slot s holds [D][C] coordinates then [C] ids (u32)
    psi::Buf slots;
    uint64_t slot_top = 0;  // slots ever handed out (bump pointer)
    psi::Buf free_stack;    // freed slots, reused before bumping
    uint64_t n_free = 0;

    // leaf directory (double-buffered for updates): records and pivots
    psi::Buf leaf[2], pkey[2], pid[2];
    int cur = 0;
    uint64_t L = 0;

    // node levels 0..h-1, level-major from the root
    psi::Buf inner;
    psi::Buf cinner, cleaf;  // packed boxes of the inner nodes and of the leaves
    bool boxes_fresh = false;  // packed boxes match the current tree
    uint64_t n_inner = 0;
    uint32_t h = 0;
    std::vector<psi::LevelInfo> lv;

    uint32_t bucket_top = ~0u;  // bucket bits of the last two-level build sort

    psi::Buf err;      // device u32 error bits
    void* pinned = nullptr;  // host readback area (4 KiB)
    psi::Sorter sorter;
    psi::Scratch scr;
    psi::Prof prof;

    uint64_t slot_words() const { return (uint64_t)(D + 1) * C; }
    psi::TreeView view() const;
};

namespace psi {

// Records launches of one kernel family between HIP events when profiling.
struct ProfScope {
    psi_index ix;
    const char* fam;
    uint64_t bytes;
    hipEvent_t a = nullptr;
    ProfScope(psi_index x, const char* f, uint64_t b) : ix(x), fam(f), bytes(b) {
        if (ix->prof.on) {
            a = ix->prof.take();
            (void)hipEventRecord(a, ix->st);
        }
    }
    ~ProfScope() {
        if (ix->prof.on) {
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
psi_status ensure_q(Buf& b, size_t need, hipStream_t st);
psi_status sort_pairs(psi_index ix, const uint64_t* kin, const uint32_t* iin, uint32_t id_base, uint64_t n,
                      bool id_digits, bool hist_ready, int* which, const char* fam, uint32_t key_shift0 = 0,
                      int key_passes = 8);
psi_status build_nodes(psi_index ix);
psi_status readback(psi_index ix, const void* dev, size_t bytes);  // into ix->pinned, waits

// updates (psi_update.hip)
psi_status do_insert(psi_index ix, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids);
psi_status do_delete(psi_index ix, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted);
psi_status do_build(psi_index ix, const uint32_t* d_pts, uint64_t n, uint32_t id_base);
psi_status encode_sort(psi_index ix, const uint32_t* d_pts, uint64_t n, uint32_t id_base, int* which);
// Processing order of a query batch (curve keys of the points or box centres
// in scr.c, input order; *order null or the positions sorted by key); latches
// ERR_RANGE for out-of-range query points.
psi_status query_order(psi_index ix, const uint32_t* d_items, uint64_t n, bool boxes, const uint32_t** order);

}  // namespace psi
