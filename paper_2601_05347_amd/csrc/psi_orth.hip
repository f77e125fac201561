// C ABI of the P-Orth tree (Sec. 3, Alg. 1): build from points sorted by
// Morton key, then kNN and range queries (kernels in k_orth.hip).
#include <cstring>
#include <new>

#include "psi_index.h"

using namespace psi;

struct psi_orth_s {
    psi_index ix = nullptr;  // stream, sort workspace, error word, timing
    psi::Buf box, link, first, pts, ids, lev, mark, lstart, llev, fkey, tcnt, toff, cnt1, base, tmp, small;
    uint64_t n = 0, N = 0, L = 0;
    uint32_t height = 0;

    psi::OrthView view() const {
        psi::OrthView v{};
        v.box = box.as<uint4>();
        v.link = link.as<uint2>();
        v.first = first.as<uint32_t>();
        v.pts = pts.as<uint4>();
        v.ids = ids.as<uint32_t>();
        v.lstart = lstart.as<uint32_t>();
        v.fkey = fkey.as<uint64_t>();
        v.N = N;
        v.L = (uint32_t)L;
        v.n = (uint32_t)n;
        return v;
    }
};

namespace {

psi_status last_launch() { return hip_ok(hipGetLastError()); }

// Copies `words` u32 from each of two device addresses into the pinned
// area (a then b) and waits.
psi_status read2(psi_index ix, const uint32_t* a, uint32_t na, const uint32_t* b, uint32_t nb) {
    psi_status s = hip_ok(hipMemcpyAsync(ix->pinned, a, na * 4, hipMemcpyDeviceToHost, ix->st));
    if (s == PSI_OK && nb)
        s = hip_ok(hipMemcpyAsync(static_cast<uint32_t*>(ix->pinned) + na, b, nb * 4, hipMemcpyDeviceToHost, ix->st));
    if (s != PSI_OK) return s;
    return hip_ok(hipStreamSynchronize(ix->st));
}

psi_status orth_build(psi_orth o, const uint32_t* d_pts, uint64_t n) {
    psi_index ix = o->ix;
    hipStream_t st = ix->st;
    psi_status s;
    o->n = o->N = o->L = 0;
    o->height = 0;
    if (n == 0) return PSI_OK;
    if ((s = ix->idkey.ensure(n * 8)) != PSI_OK) return s;
    int w = 0;
    if ((s = encode_sort(ix, d_pts, n, 0, &w)) != PSI_OK) return s;
    const uint64_t* sk = ix->sorter.k[w].as<uint64_t>();
    const uint32_t* sid = ix->sorter.i[w].as<uint32_t>();
    const uint64_t tiles = (n + ORTH_TILE - 1) / ORTH_TILE;
    if ((s = o->tcnt.ensure(tiles * 4)) != PSI_OK) return s;
    if ((s = o->toff.ensure(tiles * 4 + 4)) != PSI_OK) return s;
    if ((s = o->tmp.ensure(scan_tmp_words(n) * 4)) != PSI_OK) return s;  // scans of tiles, then of L <= n leaves
    if ((s = o->small.ensure(64)) != PSI_OK) return s;
    if ((s = o->pts.ensure(n * 16)) != PSI_OK) return s;
    if ((s = o->ids.ensure(n * 4)) != PSI_OK) return s;
    if ((s = o->mark.ensure(tiles * ORTH_TILE)) != PSI_OK) return s;
    // leaf cut: marks, points and tile counts; scan; then the leaves
    uint32_t* small = o->small.as<uint32_t>();
    {
        ProfScope ps(ix, "orth_marks", n * 30 + tiles * 4);
        launch_orth_mark(st, ix->D, sk, sid, n, ix->phi, o->mark.as<uint8_t>(), o->tcnt.as<uint32_t>(),
                         o->pts.as<uint4>(), o->ids.as<uint32_t>());
    }
    launch_scan_u32(st, o->tcnt.as<uint32_t>(), o->toff.as<uint32_t>(), tiles, small, o->tmp.as<uint32_t>());
    if ((s = last_launch()) != PSI_OK) return s;
    if ((s = read2(ix, small, 1, ix->err.as<uint32_t>(), 1)) != PSI_OK) return s;
    uint32_t h[2];
    std::memcpy(h, ix->pinned, 8);
    if (h[1] & ERR_RANGE) {  // keys of out-of-range points: no tree
        launch_fill_u32(st, ix->err.as<uint32_t>(), 1, 0u);
        (void)hipStreamSynchronize(st);
        return PSI_E_RANGE;
    }
    const uint64_t L = h[0];
    if (L == 0 || L > n) return PSI_E_INTERNAL;
    if ((s = o->lstart.ensure(L * 4)) != PSI_OK) return s;
    if ((s = o->llev.ensure(L)) != PSI_OK) return s;
    if ((s = o->fkey.ensure(L * 8)) != PSI_OK) return s;
    if ((s = o->cnt1.ensure(L * 4)) != PSI_OK) return s;
    if ((s = o->base.ensure(L * 4)) != PSI_OK) return s;
    {
        ProfScope ps(ix, "orth_marks", n + L * 21);
        launch_orth_leaves(st, sk, n, o->mark.as<uint8_t>(), o->toff.as<uint32_t>(), o->lstart.as<uint32_t>(),
                           o->llev.as<uint8_t>(), o->fkey.as<uint64_t>());
    }
    // nodes opened per leaf -> preorder positions
    launch_fill_u32(st, small, 2, 0u);
    {
        ProfScope ps(ix, "orth_nodes", L * 13);
        launch_orth_counts(st, ix->D, o->llev.as<uint8_t>(), o->fkey.as<uint64_t>(), (uint32_t)L,
                           o->cnt1.as<uint32_t>(), small + 1, ix->err.as<uint32_t>());
    }
    launch_scan_u32(st, o->cnt1.as<uint32_t>(), o->base.as<uint32_t>(), L, small, o->tmp.as<uint32_t>());
    if ((s = last_launch()) != PSI_OK) return s;
    if ((s = read2(ix, small, 2, nullptr, 0)) != PSI_OK) return s;
    std::memcpy(h, ix->pinned, 8);
    const uint64_t N = h[0];
    const uint32_t maxlev = h[1];
    // N is a 32-bit sum: it cannot have wrapped while L (maxlev + 1) < 2^32
    if (L * (maxlev + 1ull) >= (1ull << 32)) return PSI_E_CAPACITY;
    if (N < L) return PSI_E_INTERNAL;
    if ((s = o->box.ensure(N * 16)) != PSI_OK) return s;
    if ((s = o->link.ensure(N * 8)) != PSI_OK) return s;
    if ((s = o->first.ensure(N * 4)) != PSI_OK) return s;
    if ((s = o->lev.ensure(N)) != PSI_OK) return s;
    {
        ProfScope ps(ix, "orth_nodes", L * 21 + N * 29 + n * 16);
        launch_orth_nodes(st, ix->D, o->llev.as<uint8_t>(), o->fkey.as<uint64_t>(), o->lstart.as<uint32_t>(),
                          o->base.as<uint32_t>(), (uint32_t)L, (uint32_t)n, N, o->pts.as<uint4>(),
                          o->box.as<uint4>(), o->link.as<uint2>(), o->first.as<uint32_t>(),
                          o->lev.as<uint8_t>());
    }
    {
        ProfScope ps(ix, "orth_boxes", N * (uint64_t)maxlev + (N - L) * 48);
        for (uint32_t l = maxlev; l-- > 0;)
            launch_orth_boxes(st, ix->D, l, N, o->lev.as<uint8_t>(), o->box.as<uint4>(), o->link.as<uint2>());
    }
    if ((s = last_launch()) != PSI_OK) return s;
    o->n = n;
    o->N = N;
    o->L = L;
    o->height = maxlev + 1;
    return PSI_OK;
}

}  // namespace

extern "C" {

psi_status psi_orth_create(const psi_params* prm, void* hip_stream, psi_orth* out) {
    if (!prm || !out) return PSI_E_ARG;
    *out = nullptr;
    if (prm->curve != PSI_MORTON ||
        (prm->flags & ~(uint32_t)(PSI_FLAG_INPUT_ORDER | PSI_FLAG_SORT_BUCKETS | PSI_FLAG_SORT_LSD)) != 0)
        return PSI_E_ARG;
    psi_params p = *prm;
    p.fanout = 8;  // unused by the orth tree; a valid value for the shared state
    psi_orth o = new (std::nothrow) psi_orth_s;
    if (!o) return PSI_E_NOMEM;
    psi_status s = psi_create(&p, hip_stream, &o->ix);
    if (s != PSI_OK) {
        delete o;
        return s;
    }
    *out = o;
    return PSI_OK;
}

psi_status psi_orth_destroy(psi_orth o) {
    if (!o) return PSI_E_ARG;
    (void)hipStreamSynchronize(o->ix->st);
    psi_destroy(o->ix);
    delete o;
    return PSI_OK;
}

psi_status psi_orth_build(psi_orth o, const uint32_t* d_pts, uint64_t n) {
    if (!o || (n && !d_pts)) return PSI_E_ARG;
    if (n >= (1ull << 31)) return PSI_E_CAPACITY;
    if (capturing(o->ix->st)) return PSI_E_STATE;
    psi_status s = orth_build(o, d_pts, n);
    if (s != PSI_OK) {
        o->n = o->N = o->L = 0;
        o->height = 0;
    }
    return s;
}

psi_status psi_orth_knn(psi_orth o, const uint32_t* d_q, uint64_t nq, uint32_t k, uint32_t* d_ids, uint64_t* d_d2) {
    if (!o || k == 0 || k > 16 || (nq && (!d_q || !d_ids || !d_d2))) return PSI_E_ARG;
    if (nq == 0) return PSI_OK;
    psi_index ix = o->ix;
    const uint32_t* order = nullptr;
    psi_status s = query_order(ix, d_q, nq, false, &order);
    if (s != PSI_OK) return s;
    ProfScope ps(ix, "orth_knn", nq * (4ull * ix->D + 12ull * k));
    launch_orth_knn(ix->st, ix->D, o->view(), d_q, ix->scr.c.as<uint64_t>(), nq, order, k, d_ids, d_d2);
    return last_launch();
}

psi_status psi_orth_range_count(psi_orth o, const uint32_t* d_boxes, uint64_t nb, uint64_t* d_counts) {
    if (!o || (nb && (!d_boxes || !d_counts))) return PSI_E_ARG;
    if (nb == 0) return PSI_OK;
    psi_index ix = o->ix;
    const uint32_t* order = nullptr;
    psi_status s = query_order(ix, d_boxes, nb, true, &order);
    if (s != PSI_OK) return s;
    ProfScope ps(ix, "orth_range_count", nb * (8ull * ix->D + 8));
    launch_orth_range(ix->st, ix->D, o->view(), d_boxes, nb, order, d_counts, nullptr, nullptr);
    return last_launch();
}

psi_status psi_orth_range_report(psi_orth o, const uint32_t* d_boxes, uint64_t nb, const uint64_t* d_offsets,
                                 uint32_t* d_ids) {
    if (!o || (nb && (!d_boxes || !d_offsets))) return PSI_E_ARG;
    if (nb == 0) return PSI_OK;
    psi_index ix = o->ix;
    const uint32_t* order = nullptr;
    psi_status s = query_order(ix, d_boxes, nb, true, &order);
    if (s != PSI_OK) return s;
    // nothing to write without an output array (every box then reports 0 ids)
    if (!d_ids) return PSI_OK;
    ProfScope ps(ix, "orth_range_report", nb * (8ull * ix->D + 16));
    launch_orth_range(ix->st, ix->D, o->view(), d_boxes, nb, order, nullptr, d_offsets, d_ids);
    return last_launch();
}

psi_status psi_orth_sync(psi_orth o) {
    if (!o) return PSI_E_ARG;
    return psi_sync(o->ix);
}

psi_status psi_orth_shape(psi_orth o, uint64_t* h_nodes, uint64_t* h_leaves, uint32_t* h_height) {
    if (!o) return PSI_E_ARG;
    if (h_nodes) *h_nodes = o->N;
    if (h_leaves) *h_leaves = o->L;
    if (h_height) *h_height = o->height;
    return PSI_OK;
}

psi_status psi_orth_export(psi_orth o, uint32_t* d_nodes, uint32_t* d_pts) {
    if (!o) return PSI_E_ARG;
    hipStream_t st = o->ix->st;
    psi_status s = PSI_OK;
    if (d_nodes && o->N) {
        launch_orth_export(st, o->ix->D, o->box.as<uint4>(), o->link.as<uint2>(), o->N, d_nodes);
        s = last_launch();
    }
    if (s == PSI_OK && d_pts && o->n)
        s = hip_ok(hipMemcpyAsync(d_pts, o->pts.p, o->n * 16, hipMemcpyDeviceToDevice, st));
    if (s != PSI_OK) return s;
    return hip_ok(hipStreamSynchronize(st));
}

psi_status psi_orth_prof_enable(psi_orth o, int on) {
    if (!o) return PSI_E_ARG;
    return psi_prof_enable(o->ix, on);
}

psi_status psi_orth_prof_reset(psi_orth o) {
    if (!o) return PSI_E_ARG;
    return psi_prof_reset(o->ix);
}

psi_status psi_orth_prof_get(psi_orth o, const char* family, double* h_ms, uint64_t* h_launches, uint64_t* h_bytes) {
    if (!o) return PSI_E_ARG;
    return psi_prof_get(o->ix, family, h_ms, h_launches, h_bytes);
}

}  // extern "C"
