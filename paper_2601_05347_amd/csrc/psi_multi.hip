// Batched small indexes (C ABI): many independent SPaC-trees built with one
// segmented pipeline, queried with one persistent launch.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "psi_index.h"

using namespace psi;

struct psi_multi_s {
    int D = 2, curve = 0;
    uint32_t phi = 32, C = 64, B = 8;
    hipStream_t st = nullptr;
    uint32_t num = 0;
    uint32_t max_h = 0;  // the tallest index's height
    uint64_t n_total = 0, total_leaves = 0, total_inner = 0, total_tiles = 0;
    std::vector<uint64_t> pt_off;   // host copy of the point offsets
    std::vector<IdxMeta> meta_h;    // host copy of the per-index metadata
    Buf keys, k[2], i[2], hist, off, status, ctr, tiles, seg, slots, leaf, pkey, pid, inner, meta, pref, err, qtmp;
    uint32_t epoch = 0;
    void* pinned = nullptr;
    void* stage = nullptr;  // pinned staging of the build's tables
    TreeView view() const {
        TreeView t{};
        t.inner = inner.as<NodeRec>();
        t.leaf = leaf.as<NodeRec>();
        t.pkey = pkey.as<uint64_t>();
        t.slots = slots.as<uint32_t>();
        t.B = B;
        t.C = C;
        t.L = total_leaves;
        return t;
    }
    // single-index view of index s (for inspection)
    TreeView view_of(uint32_t s) const {
        TreeView t = view();
        const IdxMeta& m = meta_h[s];
        t.inner = inner.as<NodeRec>() + m.inner_base;
        t.leaf = leaf.as<NodeRec>() + m.leaf_base;
        t.pkey = pkey.as<uint64_t>() + m.leaf_base;
        t.L = m.L;
        t.h = m.h;
        return t;
    }
};

namespace {

psi_status ok(hipError_t e) { return hip_ok(e); }

psi_status multi_build(psi_multi mx, const uint64_t* d_pt_off, const uint32_t* d_pts) {
    hipStream_t st = mx->st;
    psi_status s;
    const uint32_t num = mx->num;
    mx->pt_off.assign(num + 1, 0);
    if ((s = ok(hipMemcpyAsync(mx->pt_off.data(), d_pt_off, (num + 1) * 8, hipMemcpyDeviceToHost, st))) != PSI_OK)
        return s;
    if ((s = ok(hipStreamSynchronize(st))) != PSI_OK) return s;
    const std::vector<uint64_t>& po = mx->pt_off;
    if (po[0] != 0) return PSI_E_ARG;
    for (uint32_t x = 0; x < num; ++x)
        if (po[x + 1] < po[x] || po[x + 1] - po[x] > (1ull << 24)) return PSI_E_ARG;
    const uint64_t N = po[num];
    if (N >= 0xFFFFFFFFull) return PSI_E_CAPACITY;
    mx->n_total = N;

    // tiles (never straddling an index), leaves and tree shapes, on the host
    std::vector<uint32_t> tile_seg, tile_beg, seg_first(num), seg_end(num), leaf_off(num + 1, 0);
    mx->meta_h.assign(num, IdxMeta{});
    uint64_t inner_total = 0;
    uint32_t max_h = 0;
    for (uint32_t x = 0; x < num; ++x) {
        const uint64_t n = po[x + 1] - po[x];
        seg_first[x] = (uint32_t)tile_seg.size();
        seg_end[x] = (uint32_t)po[x + 1];
        for (uint64_t b = 0; b < n; b += SORT_TILE) {
            tile_seg.push_back(x);
            tile_beg.push_back((uint32_t)(po[x] + b));
        }
        IdxMeta& m = mx->meta_h[x];
        m.n = (uint32_t)n;
        m.pt_base = (uint32_t)po[x];
        m.L = (uint32_t)((n + mx->phi - 1) / mx->phi);
        m.leaf_base = leaf_off[x];
        leaf_off[x + 1] = leaf_off[x] + m.L;
        std::vector<uint32_t> sizes;  // leaves first
        if (m.L) {
            uint32_t c = m.L;
            sizes.push_back(c);
            while (c > 1) {
                c = (c + mx->B - 1) / mx->B;
                sizes.push_back(c);
            }
        }
        m.h = sizes.empty() ? 0 : (uint32_t)sizes.size() - 1;
        if (m.h + 1 > (uint32_t)MULTI_LEVELS) return PSI_E_ARG;
        m.inner_base = (uint32_t)inner_total;
        uint32_t o = 0;
        for (uint32_t l = 0; l <= m.h && !sizes.empty(); ++l) {
            m.lvl_n[l] = sizes[m.h - l];
            m.lvl_off[l] = l < m.h ? o : 0;
            if (l < m.h) o += sizes[m.h - l];
        }
        inner_total += o;
        max_h = std::max(max_h, m.h);
    }
    mx->max_h = max_h;
    mx->total_tiles = tile_seg.size();
    mx->total_leaves = leaf_off[num];
    mx->total_inner = inner_total;
    // parents per height step, prefix over indexes
    std::vector<uint32_t> pref((size_t)max_h * (num + 1), 0);
    std::vector<uint64_t> nparents(max_h + 1, 0);
    for (uint32_t u = 1; u <= max_h; ++u) {
        uint32_t* p = pref.data() + (size_t)(u - 1) * (num + 1);
        for (uint32_t x = 0; x < num; ++x) {
            const IdxMeta& m = mx->meta_h[x];
            p[x + 1] = p[x] + (m.h >= u ? m.lvl_n[m.h - u] : 0u);
        }
        nparents[u] = p[num];
    }

    // device buffers
    const uint64_t T = std::max<uint64_t>(mx->total_tiles, 1);
    if ((s = mx->keys.ensure(std::max<uint64_t>(N, 1) * 8)) != PSI_OK) return s;
    for (int b = 0; b < 2; ++b) {
        if ((s = mx->k[b].ensure(std::max<uint64_t>(N, 1) * 8)) != PSI_OK) return s;
        if ((s = mx->i[b].ensure(std::max<uint64_t>(N, 1) * 4)) != PSI_OK) return s;
    }
    if ((s = mx->hist.ensure((uint64_t)num * 8 * RADIX * 4)) != PSI_OK) return s;
    if ((s = mx->off.ensure((uint64_t)num * 8 * RADIX * 4)) != PSI_OK) return s;
    if ((s = mx->ctr.ensure(64)) != PSI_OK) return s;
    const bool fresh_status = mx->status.bytes < T * RADIX * 8;
    if ((s = mx->status.ensure(T * RADIX * 8)) != PSI_OK) return s;
    if (fresh_status) launch_fill_u32(st, mx->status.as<uint32_t>(), mx->status.bytes / 4, 0u);
    if ((s = mx->tiles.ensure(T * 8)) != PSI_OK) return s;
    if ((s = mx->seg.ensure(((uint64_t)num * 3 + 1) * 8 + (uint64_t)(num + 1) * 4)) != PSI_OK) return s;
    if ((s = mx->slots.ensure(std::max<uint64_t>(mx->total_leaves, 1) * (mx->D + 1) * mx->C * 4)) != PSI_OK) return s;
    if ((s = mx->leaf.ensure(std::max<uint64_t>(mx->total_leaves, 1) * sizeof(NodeRec))) != PSI_OK) return s;
    if ((s = mx->pkey.ensure(std::max<uint64_t>(mx->total_leaves, 1) * 8)) != PSI_OK) return s;
    if ((s = mx->pid.ensure(std::max<uint64_t>(mx->total_leaves, 1) * 4)) != PSI_OK) return s;
    if ((s = mx->inner.ensure(std::max<uint64_t>(inner_total, 1) * sizeof(NodeRec))) != PSI_OK) return s;
    if ((s = mx->meta.ensure((uint64_t)num * sizeof(IdxMeta))) != PSI_OK) return s;
    if ((s = mx->pref.ensure(std::max<size_t>(pref.size(), 1) * 4)) != PSI_OK) return s;

    uint32_t* d_tile_seg = mx->tiles.as<uint32_t>();
    uint32_t* d_tile_beg = d_tile_seg + T;
    uint32_t* d_seg_first = mx->seg.as<uint32_t>();
    uint32_t* d_seg_end = d_seg_first + num;
    uint32_t* d_leaf_off = d_seg_end + num;
    uint64_t* d_seg_begin = reinterpret_cast<uint64_t*>(mx->seg.as<char>() + (((uint64_t)num * 3 + 1) * 4 + 7) / 8 * 8);
    // The host-built tables go through one pinned staging block, copied on the
    // stream without waiting; the block lives until the index is destroyed
    // (which waits for the stream).
    struct Piece {
        void* dst;
        const void* src;
        size_t bytes;
    };
    const Piece pieces[] = {{d_tile_seg, tile_seg.data(), tile_seg.size() * 4},
                            {d_tile_beg, tile_beg.data(), tile_beg.size() * 4},
                            {d_seg_first, seg_first.data(), (size_t)num * 4},
                            {d_seg_end, seg_end.data(), (size_t)num * 4},
                            {d_leaf_off, leaf_off.data(), (size_t)(num + 1) * 4},
                            {d_seg_begin, po.data(), (size_t)num * 8},
                            {mx->meta.p, mx->meta_h.data(), (size_t)num * sizeof(IdxMeta)},
                            {mx->pref.p, pref.data(), pref.size() * 4}};
    size_t stage_bytes = 0;
    for (const Piece& pc : pieces) stage_bytes += (pc.bytes + 255) / 256 * 256;
    if (mx->stage) (void)hipHostFree(mx->stage);
    mx->stage = nullptr;
    if ((s = ok(hipHostMalloc(&mx->stage, std::max<size_t>(stage_bytes, 256), hipHostMallocDefault))) != PSI_OK) {
        mx->stage = nullptr;
        return s;
    }
    char* h = static_cast<char*>(mx->stage);
    for (const Piece& pc : pieces) {
        if (pc.bytes == 0) continue;
        std::memcpy(h, pc.src, pc.bytes);
        if ((s = ok(hipMemcpyAsync(pc.dst, h, pc.bytes, hipMemcpyHostToDevice, st))) != PSI_OK) return s;
        h += (pc.bytes + 255) / 256 * 256;
    }
    if (N == 0) return PSI_OK;

    SegTiles sg{d_tile_seg, d_tile_beg, d_seg_first, d_seg_end, 8 * RADIX};
    launch_fill_u32(st, mx->hist.as<uint32_t>(), (uint64_t)num * 8 * RADIX, 0u);
    launch_encode_hist_seg(st, mx->D, mx->curve, d_pts, mx->total_tiles, sg, mx->keys.as<uint64_t>(),
                           mx->hist.as<uint32_t>(), mx->err.as<uint32_t>());
    launch_seg_digit_offsets(st, num, mx->hist.as<uint32_t>(), d_seg_begin, mx->off.as<uint32_t>());
    launch_fill_u32(st, mx->ctr.as<uint32_t>(), 16, 0u);
    const uint64_t* ksrc = mx->keys.as<uint64_t>();
    const uint32_t* isrc = nullptr;
    for (int p = 0; p < 8; ++p) {
        const int dst = p & 1;
        if (++mx->epoch >= (1u << 30)) {
            mx->epoch = 1;
            launch_fill_u32(st, mx->status.as<uint32_t>(), mx->status.bytes / 4, 0u);
        }
        launch_onesweep(st, p == 0, false, ksrc, isrc, 0, mx->k[dst].as<uint64_t>(), mx->i[dst].as<uint32_t>(), N,
                        8 * p, mx->off.as<uint32_t>() + p * RADIX, mx->status.as<uint64_t>(),
                        mx->ctr.as<uint32_t>() + p, mx->epoch, mx->err.as<uint32_t>(), &sg, mx->total_tiles);
        ksrc = mx->k[dst].as<uint64_t>();
        isrc = mx->i[dst].as<uint32_t>();
    }
    launch_build_leaves_seg(st, mx->D, mx->curve, num, mx->total_leaves, d_leaf_off, mx->meta.as<IdxMeta>(),
                            mx->k[1].as<uint64_t>(), mx->i[1].as<uint32_t>(), mx->C, mx->slots.as<uint32_t>(),
                            mx->pkey.as<uint64_t>(), mx->pid.as<uint32_t>(), mx->leaf.as<NodeRec>());
    for (uint32_t u = 1; u <= max_h; ++u)
        launch_node_step_seg(st, mx->D, num, nparents[u], u, mx->pref.as<uint32_t>() + (size_t)(u - 1) * (num + 1),
                             mx->meta.as<IdxMeta>(), mx->leaf.as<NodeRec>(), mx->inner.as<NodeRec>(), mx->B);
    return ok(hipGetLastError());
}

}  // namespace

extern "C" {

psi_status psi_multi_build(const psi_params* prm, void* hip_stream, uint32_t num, const uint64_t* d_pt_off,
                           const uint32_t* d_pts, psi_multi* out) {
    if (!prm || !out || num == 0 || !d_pt_off) return PSI_E_ARG;
    *out = nullptr;
    if ((prm->dim != 2 && prm->dim != 3) || prm->curve > 1 || prm->leaf_size < 2 || prm->leaf_size > 32 ||
        prm->fanout < 2 || prm->fanout > 32)
        return PSI_E_ARG;
    psi_multi mx = new (std::nothrow) psi_multi_s;
    if (!mx) return PSI_E_NOMEM;
    mx->D = (int)prm->dim;
    mx->curve = (int)prm->curve;
    mx->phi = prm->leaf_size;
    mx->C = (2 * prm->leaf_size + 3) & ~3u;
    mx->B = prm->fanout;
    mx->num = num;
    mx->st = static_cast<hipStream_t>(hip_stream);
    psi_status s = mx->err.ensure(64);
    if (s == PSI_OK) s = hip_ok(hipHostMalloc(&mx->pinned, 4096, hipHostMallocDefault));
    if (s == PSI_OK) launch_fill_u32(mx->st, mx->err.as<uint32_t>(), 16, 0u);
    if (s == PSI_OK) s = multi_build(mx, d_pt_off, d_pts);
    if (s != PSI_OK) {
        (void)hipStreamSynchronize(mx->st);
        if (mx->pinned) (void)hipHostFree(mx->pinned);
        if (mx->stage) (void)hipHostFree(mx->stage);
        delete mx;
        return s;
    }
    *out = mx;
    return PSI_OK;
}

psi_status psi_multi_destroy(psi_multi mx) {
    if (!mx) return PSI_E_ARG;
    (void)hipStreamSynchronize(mx->st);
    if (mx->pinned) (void)hipHostFree(mx->pinned);
    if (mx->stage) (void)hipHostFree(mx->stage);
    delete mx;
    return PSI_OK;
}

psi_status psi_multi_knn(psi_multi mx, const uint64_t* d_q_off, const uint32_t* d_q, uint32_t k, uint32_t* d_ids,
                         uint64_t* d_d2) {
    if (!mx || !d_q_off || !d_q || !d_ids || !d_d2) return PSI_E_ARG;
    if (k != 1 && k != 2 && k != 4 && k != 8 && k != 10 && k != 16) return PSI_E_ARG;
    psi_status s;
    const size_t need = ((uint64_t)mx->num + 1 + scan_tmp_words(mx->num) + 64) * 4;
    if (need > mx->qtmp.bytes) {
        if (capturing(mx->st)) return PSI_E_STATE;  // a captured call cannot allocate
        if ((s = mx->qtmp.ensure(need)) != PSI_OK) return s;
    }
    uint32_t* pref = mx->qtmp.as<uint32_t>();
    uint32_t* work = pref + mx->num + 1;
    uint32_t* tmp = work + 16;
    launch_multi_knn(mx->st, mx->D, mx->curve, mx->view(), mx->meta.as<IdxMeta>(), mx->num, d_q_off, d_q, pref, work, k,
                     mx->max_h, d_ids, d_d2, tmp, mx->err.as<uint32_t>());
    return hip_ok(hipGetLastError());
}

psi_status psi_multi_sync(psi_multi mx) {
    if (!mx) return PSI_E_ARG;
    psi_status s = hip_ok(hipMemcpyAsync(mx->pinned, mx->err.p, 4, hipMemcpyDeviceToHost, mx->st));
    if (s == PSI_OK) s = hip_ok(hipStreamSynchronize(mx->st));
    if (s != PSI_OK) return s;
    uint32_t e = 0;
    std::memcpy(&e, mx->pinned, 4);
    if (e) {
        launch_fill_u32(mx->st, mx->err.as<uint32_t>(), 1, 0u);
        (void)hipStreamSynchronize(mx->st);
        return (e & ERR_RANGE) ? PSI_E_RANGE : PSI_E_INTERNAL;
    }
    return PSI_OK;
}

psi_status psi_multi_shape(psi_multi mx, uint32_t index, uint64_t* h_n_leaves, uint32_t* h_height,
                           uint64_t* h_level_sizes) {
    if (!mx || index >= mx->num || !h_n_leaves || !h_height) return PSI_E_ARG;
    const IdxMeta& m = mx->meta_h[index];
    *h_n_leaves = m.L;
    *h_height = m.h;
    if (h_level_sizes && m.L)
        for (uint32_t l = 0; l <= m.h; ++l) h_level_sizes[l] = m.lvl_n[l];
    return PSI_OK;
}

psi_status psi_multi_export_structure(psi_multi mx, uint32_t index, uint64_t* d_piv_key, uint32_t* d_piv_id,
                                      uint32_t* d_leaf_cnt, uint32_t* d_leaf_lo, uint32_t* d_leaf_hi,
                                      uint32_t* d_node_lo, uint32_t* d_node_hi, uint64_t* d_node_cnt) {
    if (!mx || index >= mx->num) return PSI_E_ARG;
    const IdxMeta& m = mx->meta_h[index];
    if (m.L == 0) return PSI_OK;
    uint64_t n_inner = 0;
    for (uint32_t l = 0; l < m.h; ++l) n_inner += m.lvl_n[l];
    launch_export_structure(mx->st, mx->D, mx->view_of(index), n_inner, mx->pkey.as<uint64_t>() + m.leaf_base,
                            mx->pid.as<uint32_t>() + m.leaf_base, d_piv_key, d_piv_id, d_leaf_cnt, d_leaf_lo,
                            d_leaf_hi, d_node_lo, d_node_hi, d_node_cnt);
    return hip_ok(hipGetLastError());
}

psi_status psi_multi_export(psi_multi mx, uint64_t* d_keys, uint32_t* d_ids, uint32_t* d_pts) {
    if (!mx) return PSI_E_ARG;
    if (mx->total_leaves == 0) return PSI_OK;
    psi_status s;
    const uint64_t L = mx->total_leaves;
    if ((s = mx->qtmp.ensure(((L + 1) * 2 + 2 * L + scan_tmp_words(L) + 8) * 8)) != PSI_OK) return s;
    uint64_t* off = mx->qtmp.as<uint64_t>();
    launch_leaf_offsets(mx->st, mx->leaf.as<NodeRec>(), L, off, off + L + 1);
    launch_export_sorted(mx->st, mx->D, mx->curve, mx->view(), off, d_keys, d_ids, d_pts);
    return hip_ok(hipGetLastError());
}

}  // extern "C"
