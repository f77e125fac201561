// C ABI of the P-Orth tree (Sec. 3, Alg. 1): build from points sorted by
// Morton key, then kNN and range queries (kernels in k_orth.hip).
#include <cstring>
#include <new>

#include "psi_index.h"

using namespace psi;

struct psi_orth_s {
    psi_index ix = nullptr;  // stream, sort workspace, error word, timing
    psi::Buf box, link, first, pts, ids, lev, lbox, mark, lstart, llev, fkey, tcnt, toff, cnt1, base, tmp, small;
    psi::Buf alive;             // live bit per id ever handed out
    psi::Buf mk, mi, place, hist, hscan, flag;  // batch updates: the new set's sorted pairs
    uint64_t n = 0, N = 0, L = 0;
    uint32_t height = 0;
    uint32_t next_id = 0;

    psi::OrthView view() const {
        psi::OrthView v{};
        v.box = box.as<uint4>();
        v.link = link.as<uint2>();
        v.first = first.as<uint32_t>();
        v.pts = pts.as<uint4>();
        v.ids = ids.as<uint32_t>();
        v.lstart = lstart.as<uint32_t>();
        v.fkey = fkey.as<uint64_t>();
        v.llev = llev.as<uint8_t>();
        v.base = base.as<uint32_t>();
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

// The tree of the n pairs (sk, sid) sorted by (Morton key, id): leaf cut,
// points, nodes and boxes. Reports PSI_E_RANGE (no tree) if an encode of the
// pairs' points latched a range error.
psi_status orth_cut(psi_orth o, const uint64_t* sk, const uint32_t* sid, uint64_t n) {
    psi_index ix = o->ix;
    hipStream_t st = ix->st;
    psi_status s;
    o->n = o->N = o->L = 0;
    o->height = 0;
    if (n == 0) return PSI_OK;
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
    // the sort's bucket bits, the next build's guess (the stream is idle)
    uint32_t top = ~0u;
    if (hipMemcpy(&top, &ix->dt()->sort_top, 4, hipMemcpyDeviceToHost) == hipSuccess) ix->bucket_top = top;
    else (void)hipGetLastError();
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
    if ((s = o->lbox.ensure(L * 16)) != PSI_OK) return s;
    {
        ProfScope ps(ix, "orth_marks", n * 9 + L * 37);
        launch_orth_leaves(st, ix->D, sk, n, o->mark.as<uint8_t>(), o->toff.as<uint32_t>(), o->lstart.as<uint32_t>(),
                           o->llev.as<uint8_t>(), o->fkey.as<uint64_t>(), o->lbox.as<uint4>());
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
        ProfScope ps(ix, "orth_nodes", L * 37 + N * 29);
        launch_orth_nodes(st, ix->D, o->llev.as<uint8_t>(), o->fkey.as<uint64_t>(), o->lstart.as<uint32_t>(),
                          o->base.as<uint32_t>(), (uint32_t)L, (uint32_t)n, N, o->lbox.as<uint4>(),
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

psi_status orth_build(psi_orth o, const uint32_t* d_pts, uint64_t n) {
    psi_index ix = o->ix;
    psi_status s;
    o->n = o->N = o->L = 0;
    o->height = 0;
    o->next_id = 0;
    if (n == 0) return PSI_OK;
    if ((s = ix->idkey.ensure(n * 8)) != PSI_OK) return s;
    int w = 0;
    if ((s = encode_sort(ix, d_pts, n, ix->idkey.as<uint64_t>(), 0, &w)) != PSI_OK) return s;
    if ((s = o->alive.ensure((n + 31) / 32 * 4)) != PSI_OK) return s;
    launch_orth_alive(ix->st, o->alive.as<uint32_t>(), 0, (uint32_t)n);
    if ((s = orth_cut(o, ix->sorter.k[w].as<uint64_t>(), ix->sorter.i[w].as<uint32_t>(), n)) != PSI_OK) return s;
    o->next_id = (uint32_t)n;
    return PSI_OK;
}

// Insert: sort the batch, merge it into the old order, cut the tree again.
psi_status orth_insert(psi_orth o, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids) {
    psi_index ix = o->ix;
    hipStream_t st = ix->st;
    psi_status s;
    const uint64_t n = o->n, id0 = o->next_id;
    // the id table keeps every id's key (deletes look points up by it)
    if ((s = ix->idkey.grow_keep((id0 + m) * 8, id0 * 8, st)) != PSI_OK) return s;
    int w = 0;
    if ((s = encode_sort(ix, d_pts, m, ix->idkey.as<uint64_t>() + id0, (uint32_t)id0, &w)) != PSI_OK) return s;
    if ((s = read2(ix, ix->err.as<uint32_t>(), 1, nullptr, 0)) != PSI_OK) return s;
    uint32_t e = 0;
    std::memcpy(&e, ix->pinned, 4);
    if (e & ERR_RANGE) {  // nothing inserted, the tree unchanged
        launch_fill_u32(st, ix->err.as<uint32_t>(), 1, 0u);
        (void)hipStreamSynchronize(st);
        return PSI_E_RANGE;
    }
    const uint64_t* bk = ix->sorter.k[w].as<uint64_t>();
    const uint32_t* bid = ix->sorter.i[w].as<uint32_t>();
    if ((s = o->mk.ensure((n + m) * 8)) != PSI_OK) return s;
    if ((s = o->mi.ensure((n + m) * 4)) != PSI_OK) return s;
    if ((s = o->place.ensure(m * 4)) != PSI_OK) return s;
    if ((s = o->hist.ensure((n + 1) * 4)) != PSI_OK) return s;
    if ((s = o->hscan.ensure((n + 1) * 4)) != PSI_OK) return s;
    if ((s = o->tmp.ensure(scan_tmp_words(n + m + 1) * 4)) != PSI_OK) return s;
    {
        ProfScope ps(ix, "orth_merge", m * 16 * 20 + n * 44);
        launch_fill_u32(st, o->hist.as<uint32_t>(), n + 1, 0u);
        launch_orth_place(st, ix->D, o->pts.as<uint4>(), n, bk, m, o->place.as<uint32_t>(), o->hist.as<uint32_t>());
        launch_scan_u32(st, o->hist.as<uint32_t>(), o->hscan.as<uint32_t>(), n, nullptr, o->tmp.as<uint32_t>());
        launch_orth_merge(st, ix->D, o->pts.as<uint4>(), n, o->hist.as<uint32_t>(), o->hscan.as<uint32_t>(), bk, bid,
                          o->place.as<uint32_t>(), m, o->mk.as<uint64_t>(), o->mi.as<uint32_t>());
    }
    if (d_new_ids) launch_iota_u32(st, d_new_ids, m, (uint32_t)id0);
    if ((s = o->alive.grow_keep((id0 + m + 31) / 32 * 4, (id0 + 31) / 32 * 4, st)) != PSI_OK) return s;
    launch_orth_alive(st, o->alive.as<uint32_t>(), (uint32_t)id0, (uint32_t)(id0 + m));
    if ((s = last_launch()) != PSI_OK) return s;
    o->next_id = (uint32_t)(id0 + m);
    // the cut may grow the point arrays the merge read: let the merge finish
    if ((s = hip_ok(hipStreamSynchronize(st))) != PSI_OK) return s;
    return orth_cut(o, o->mk.as<uint64_t>(), o->mi.as<uint32_t>(), n + m);
}

// Delete: clear the ids' live bits and the keep flags of their points,
// compact the old order, cut the tree again.
psi_status orth_delete(psi_orth o, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted) {
    psi_index ix = o->ix;
    hipStream_t st = ix->st;
    psi_status s;
    const uint64_t n = o->n;
    if ((s = o->small.ensure(64)) != PSI_OK) return s;
    if ((s = o->flag.ensure(std::max<uint64_t>(n, 1) * 4)) != PSI_OK) return s;
    unsigned long long* removed = reinterpret_cast<unsigned long long*>(o->small.as<uint32_t>() + 8);
    launch_orth_put64(st, removed, 0ull);
    launch_fill_u32(st, o->flag.as<uint32_t>(), n, 1u);
    if (m && o->next_id)
        launch_orth_kill(st, ix->D, d_ids, m, o->next_id, o->alive.as<uint32_t>(), ix->idkey.as<uint64_t>(),
                         o->pts.as<uint4>(), n, o->flag.as<uint32_t>(), removed, ix->err.as<uint32_t>());
    if ((s = last_launch()) != PSI_OK) return s;
    if ((s = read2(ix, reinterpret_cast<const uint32_t*>(removed), 2, nullptr, 0)) != PSI_OK) return s;
    uint64_t r = 0;
    std::memcpy(&r, ix->pinned, 8);
    if (d_ndeleted) launch_orth_put64(st, reinterpret_cast<unsigned long long*>(d_ndeleted), r);
    if (r == 0) return last_launch();
    if (r > n) return PSI_E_INTERNAL;
    if ((s = o->mk.ensure((n - r) * 8 + 8)) != PSI_OK) return s;
    if ((s = o->mi.ensure((n - r) * 4 + 4)) != PSI_OK) return s;
    if ((s = o->hscan.ensure(n * 4)) != PSI_OK) return s;
    if ((s = o->tmp.ensure(scan_tmp_words(n) * 4)) != PSI_OK) return s;
    {
        ProfScope ps(ix, "orth_merge", n * 32);
        launch_scan_u32(st, o->flag.as<uint32_t>(), o->hscan.as<uint32_t>(), n, nullptr, o->tmp.as<uint32_t>());
        launch_orth_compact(st, ix->D, o->pts.as<uint4>(), n, o->flag.as<uint32_t>(), o->hscan.as<uint32_t>(),
                            o->mk.as<uint64_t>(), o->mi.as<uint32_t>());
    }
    if ((s = last_launch()) != PSI_OK) return s;
    return orth_cut(o, o->mk.as<uint64_t>(), o->mi.as<uint32_t>(), n - r);
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
    // an error latched by an earlier call (a query's out-of-range point) is
    // reported here, not taken for this build's
    psi_status s = psi_sync(o->ix);
    if (s != PSI_OK) return s;
    s = orth_build(o, d_pts, n);
    if (s != PSI_OK) {
        o->n = o->N = o->L = 0;
        o->height = 0;
    }
    return s;
}

psi_status psi_orth_batch_insert(psi_orth o, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids) {
    if (!o || (m && !d_pts)) return PSI_E_ARG;
    if (capturing(o->ix->st)) return PSI_E_STATE;
    if ((uint64_t)o->next_id + m > 0xFFFFFFFFull || o->n + m >= (1ull << 31)) return PSI_E_CAPACITY;
    if (m == 0) return PSI_OK;
    psi_status s = psi_sync(o->ix);
    if (s != PSI_OK) return s;
    s = orth_insert(o, d_pts, m, d_new_ids);
    if (s != PSI_OK && s != PSI_E_RANGE) {  // an empty tree, ids from 0 again
        o->n = o->N = o->L = 0;
        o->height = 0;
        o->next_id = 0;
    }
    return s;
}

psi_status psi_orth_batch_delete(psi_orth o, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted) {
    if (!o || (m && !d_ids)) return PSI_E_ARG;
    if (capturing(o->ix->st)) return PSI_E_STATE;
    psi_status s = psi_sync(o->ix);
    if (s != PSI_OK) return s;
    s = orth_delete(o, d_ids, m, d_ndeleted);
    if (s != PSI_OK) {  // an empty tree, ids from 0 again
        o->n = o->N = o->L = 0;
        o->height = 0;
        o->next_id = 0;
    }
    return s;
}

psi_status psi_orth_size(psi_orth o, uint64_t* h_n_live, uint32_t* h_next_id) {
    if (!o) return PSI_E_ARG;
    if (h_n_live) *h_n_live = o->n;
    if (h_next_id) *h_next_id = o->next_id;
    return PSI_OK;
}

psi_status psi_orth_knn(psi_orth o, const uint32_t* d_q, uint64_t nq, uint32_t k, uint32_t* d_ids, uint64_t* d_d2) {
    if (!o || k == 0 || k > 128 || (nq && (!d_q || !d_ids || !d_d2))) return PSI_E_ARG;
    if (nq == 0) return PSI_OK;
    psi_index ix = o->ix;
    const uint32_t* order = nullptr;
    psi_status s = query_order(ix, d_q, nq, false, &order);
    if (s != PSI_OK) return s;
    ProfScope ps(ix, "orth_knn", nq * (4ull * ix->D + 12ull * k));
    launch_orth_knn(ix->st, ix->D, o->view(), d_q, ix->qkeys.as<uint64_t>(), nq, order, k, d_ids, d_d2);
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
