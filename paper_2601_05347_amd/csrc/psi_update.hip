// Batch insert (Alg. 4) and batch delete (Sec. 4.2): host orchestration.
//
// Both calls sort the batch's (key, id) pairs, route them to leaves and
// change the touched leaves. When no leaf is re-cut the directory is updated
// in place; otherwise a new directory is written into the other buffer:
// untouched leaves are copied, re-cut leaves get fresh slots, and the freed
// slots go to a free stack reused by later updates. Node levels are rebuilt
// over the new directory at the end. The host never learns the outcome
// before returning: it reserves room for the worst case the batch size
// allows, and the device takes every count (runs, pieces, slots, the new
// leaf count) from the counters the plan kernels leave behind.
#include <algorithm>
#include <cstring>
#include <functional>

#include "psi_index.h"
#include "psi_update.h"

namespace psi {

namespace {

// Carves 256-byte aligned arrays out of one scratch buffer.
struct Carver {
    char* base = nullptr;
    size_t off = 0;
    template <class T> T* take(uint64_t n) {
        T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += (std::max<uint64_t>(n, 1) * sizeof(T) + 255) & ~size_t(255);
        return p;
    }
};

psi_status launched() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PSI_OK : PSI_E_HIP;
}

uint64_t dir_capacity(psi_index ix) {
    uint64_t c = ~0ull;
    for (int b = 0; b < 2; ++b)
        c = std::min(c, std::min(ix->leaf[b].bytes / sizeof(NodeRec), std::min(ix->pkey[b].bytes / 8, ix->pid[b].bytes / 4)));
    return c;
}

// Most leaves whose node levels and packed boxes fit the node buffers.
uint64_t node_capacity(psi_index ix) {
    auto fits = [&](uint64_t L) {
        uint64_t inner = 0;
        for (uint64_t n = L; n > 1;) {
            n = (n + ix->B - 1) / ix->B;
            inner += n;
        }
        inner = std::max<uint64_t>(inner, 1);
        return inner * sizeof(NodeRec) <= ix->inner.bytes && inner * 16 <= ix->cinner.bytes &&
               std::max<uint64_t>(L, 1) * 16 <= ix->cleaf.bytes;
    };
    uint64_t lo = 0, hi = ix->cleaf.bytes / 16;
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) / 2;
        if (fits(mid)) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Capacities of the buffers an update writes through computed indices;
// Lg leaves covered by its per-leaf grids, Lc by its node grids.
Caps caps_of(psi_index ix, uint64_t alloc, uint64_t Lg, uint64_t Lc) {
    Caps c;
    c.leaves = std::min(dir_capacity(ix), Lc);
    c.slots = ix->slots.bytes / (ix->slot_words() * 4);
    c.frees = ix->free_stack.bytes / 4;
    c.alloc = alloc;
    c.lgrid = Lg;
    c.err = ix->err.as<uint32_t>();
    c.dirs = dirs_of(ix);
    return c;
}

// Leaf coverage of an update's grids. Eagerly: the bounds of the state
// (Lb before, L_cap after). Under graph capture the update may replay after
// the index has grown, so its grids cover as many leaves as the buffers
// already hold (scratch(L): the scratch bytes an update over L leaves
// needs); a replay finding more is refused on the device.
psi_status grid_leaves(psi_index ix, uint64_t Lb, uint64_t L_cap, const std::function<size_t(uint64_t)>& scratch,
                       uint64_t* Lg, uint64_t* Lc) {
    // at least one entry: every per-leaf launch then has a grid (an empty
    // index reads L = 0 on the device and does nothing)
    Lb = std::max<uint64_t>(Lb, 1);
    *Lg = Lb;
    *Lc = L_cap;
    if (!capturing(ix->st)) return PSI_OK;
    uint64_t lo = Lb, hi = std::max(Lb, dir_capacity(ix));
    if (scratch(lo) > ix->scr.a.bytes) return PSI_E_STATE;
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) / 2;
        if (scratch(mid) <= ix->scr.a.bytes) lo = mid;
        else hi = mid - 1;
    }
    *Lg = lo;
    *Lc = std::max(L_cap, std::min(dir_capacity(ix), node_capacity(ix)));
    return PSI_OK;
}

struct InsArrays {
    uint32_t* ctr;
    uint64_t* keys;
    uint32_t *leaf_of, *flag, *ridx, *run_leaf, *run_beg, *rpieces, *rchunks, *rsplit, *piece_off, *chunk_off,
        *free_off, *pieces, *newpos, *tmp, *slot_alloc, *piece_pos;
};

// Scratch of an insert of m points over (at most) L leaves.
InsArrays carve_ins(Carver& c, uint64_t m, uint64_t L, uint64_t A_max) {
    InsArrays a;
    a.ctr = c.take<uint32_t>(16);
    a.keys = c.take<uint64_t>(m);
    a.leaf_of = c.take<uint32_t>(m);
    a.flag = c.take<uint32_t>(m);
    a.ridx = c.take<uint32_t>(m);
    a.run_leaf = c.take<uint32_t>(m);
    a.run_beg = c.take<uint32_t>(m);
    a.rpieces = c.take<uint32_t>(m);
    a.rchunks = c.take<uint32_t>(m);
    a.rsplit = c.take<uint32_t>(m);
    a.piece_off = c.take<uint32_t>(m + 1);
    a.chunk_off = c.take<uint32_t>(m + 1);
    a.free_off = c.take<uint32_t>(m + 1);
    a.pieces = c.take<uint32_t>(L);
    a.newpos = c.take<uint32_t>(L + 1);
    a.tmp = c.take<uint32_t>(SCAN_MULTI * scan_tmp_words(std::max<uint64_t>(m, L)) + 4);
    a.slot_alloc = c.take<uint32_t>(A_max);
    a.piece_pos = c.take<uint32_t>(A_max);
    return a;
}

struct DelArrays {
    uint32_t* ctr;
    uint64_t* dk;
    uint32_t *di, *flag, *ci, *leaf_of, *ridx, *run_leaf, *run_beg;
    uint32_t *cnt, *cum, *start, *gidx, *grp_first, *gpieces, *gchunks, *galloc, *gfree, *gchanged, *gpos, *chunk_off,
        *alloc_off, *free_off, *tmp, *slot_alloc, *piece_pos;
};

// Scratch of a delete of m ids over (at most) L leaves.
DelArrays carve_del(Carver& c, uint64_t m, uint64_t L, uint64_t A_max) {
    DelArrays a;
    a.ctr = c.take<uint32_t>(16);
    a.dk = c.take<uint64_t>(m);
    a.di = c.take<uint32_t>(m);
    a.flag = c.take<uint32_t>(m);
    a.ci = nullptr;  // the sorted ids (the sorter's buffer)
    a.leaf_of = c.take<uint32_t>(m);
    a.ridx = c.take<uint32_t>(m);
    a.run_leaf = c.take<uint32_t>(m);
    a.run_beg = c.take<uint32_t>(m);
    a.cnt = c.take<uint32_t>(L);
    a.cum = c.take<uint32_t>(L + 1);
    a.start = c.take<uint32_t>(L);
    a.gidx = c.take<uint32_t>(L);
    a.grp_first = c.take<uint32_t>(L);
    a.gpieces = c.take<uint32_t>(L);
    a.gchunks = c.take<uint32_t>(L);
    a.galloc = c.take<uint32_t>(L);
    a.gfree = c.take<uint32_t>(L);
    a.gchanged = c.take<uint32_t>(L);
    a.gpos = c.take<uint32_t>(L + 1);
    a.chunk_off = c.take<uint32_t>(L + 1);
    a.alloc_off = c.take<uint32_t>(L + 1);
    a.free_off = c.take<uint32_t>(L + 1);
    a.tmp = c.take<uint32_t>(SCAN_MULTI * scan_tmp_words(std::max<uint64_t>(m, L)) + 4);
    a.slot_alloc = c.take<uint32_t>(A_max);
    a.piece_pos = c.take<uint32_t>(A_max);
    return a;
}

// Room for an update whose result may hold up to L_cap leaves, A_max new
// slots and F_max more free-stack entries, given the bounds u of the state
// before it.
psi_status reserve(psi_index ix, const Bounds& u, uint64_t L_cap, uint64_t A_max, uint64_t F_max) {
    psi_status s;
    if ((s = ensure_dirs(ix, L_cap)) != PSI_OK) return s;
    if ((s = grow_keep_q(ix, ix->slots, std::max<uint64_t>(u.slot_top + A_max, 1) * ix->slot_words() * 4)) != PSI_OK)
        return s;
    return grow_keep_q(ix, ix->free_stack, (u.n_free + F_max + 1) * 4);
}

}  // namespace

// Batch insert, queued without waiting. The bounds of the present state
// size every buffer and grid; the kernels read the true sizes from the
// device state and the counters, a one-thread check rejects a batch with an
// out-of-range coordinate (or one that would not fit) before any leaf is
// written, and a one-thread commit publishes the new state.
psi_status do_insert(psi_index ix, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids, hipEvent_t before_apply) {
    psi_status s;
    hipStream_t st = ix->st;
    Bounds u;
    if ((s = bounds(ix, &u)) != PSI_OK) return s;
    ++ix->gen;
    ProfScope ps(ix, "update", 0);
    const uint32_t phi = ix->phi;
    const uint64_t Lb = u.L;
    // A re-cut leaf held at most 2 phi entries and took r_i of the batch: it
    // becomes at most 3 + r_i / phi pieces. Hence at most min(L, m) re-cut
    // leaves, 3 min(L, m) + m / phi new slots and leaves, and chunks of
    // UPD_CHUNK outputs over at most 2 phi min(L, m) + m entries.
    const uint64_t Fm = std::min(Lb, m);
    const uint64_t A_max = 3 * Fm + m / phi + 2;
    const uint64_t L_cap = Lb + 2 * Fm + m / phi + 2;
    const uint64_t NCH_max = Fm + (2 * (uint64_t)phi * Fm + m) / UPD_CHUNK + 2;
    if ((s = reserve(ix, u, L_cap, A_max, Fm)) != PSI_OK) return s;
    if ((s = grow_keep_q(ix, ix->idkey, (u.next_id + m) * 8)) != PSI_OK) return s;
    Sorter& S = ix->sorter;
    if ((s = ensure_q(ix, S.hist, MAX_PASSES * RADIX * 4)) != PSI_OK) return s;

    auto need = [&](uint64_t L) {
        Carver c;
        carve_ins(c, m, L, A_max);
        return c.off;
    };
    uint64_t Lg = Lb, Lc = L_cap;
    if ((s = ensure_q(ix, ix->scr.a, need(std::max<uint64_t>(Lb, 1)))) != PSI_OK) return s;
    if ((s = grid_leaves(ix, Lb, L_cap, need, &Lg, &Lc)) != PSI_OK) return s;
    Carver real;
    real.base = static_cast<char*>(ix->scr.a.p);
    const InsArrays a = carve_ins(real, m, Lg, A_max);
    const Caps cap = caps_of(ix, A_max, Lg, Lc);
    const uint64_t id_cap = ix->idkey.bytes / 8;
    DevTree* dt = ix->dt();

    launch_fill_u32(st, a.ctr, 16, 0u);
    launch_fill_u32(st, S.hist.as<uint32_t>(), 8 * RADIX, 0u);
    // keys of the batch (a coordinate out of range flags ctr[9]), then the
    // pairs (key, position) sorted; positions become ids once the device
    // has checked the batch
    launch_encode_hist(st, ix->D, ix->curve, d_pts, m, a.keys, S.hist.as<uint32_t>(), a.ctr + 9);
    int w = 0;
    if ((s = sort_pairs(ix, a.keys, nullptr, 0, m, false, true, &w, "radix_update")) != PSI_OK) return s;
    const uint64_t* bk = S.k[w].as<uint64_t>();
    uint32_t* bi = S.i[w].as<uint32_t>();
    st_ins_ids(st, dt, a.keys, m, ix->idkey.as<uint64_t>(), id_cap, bi, d_new_ids, a.ctr);
    upd_route(st, bk, bi, m, nullptr, dt, cap.dirs, a.leaf_of);
    upd_runs(st, a.leaf_of, m, nullptr, a.flag, a.ridx, a.run_leaf, a.run_beg, a.ctr + 1, a.tmp);
    upd_ins_plan(st, a.run_leaf, a.run_beg, a.ctr, m, dt, cap.dirs, phi, a.rpieces, a.rchunks, a.rsplit);
    ScanSet sc{{a.rpieces, a.rchunks, a.rsplit, nullptr},
               {a.piece_off, a.chunk_off, a.free_off, nullptr},
               {a.ctr + 3, a.ctr + 4, a.ctr + 5, nullptr},
               {m, m, m, 0}};
    launch_scan_multi(st, sc, 3, a.tmp);
    // apply, reject, or (empty index) build the batch as a fresh tree
    st_ins_check(st, dt, a.ctr, m, phi, id_cap, cap);
    // new directory positions when leaves are re-cut (ctr[3] > 0): exclusive
    // scan of the per-leaf piece counts
    if (before_apply && (s = hip_ok(hipStreamWaitEvent(st, before_apply, 0))) != PSI_OK) return s;
    st_fill_gated(st, a.pieces, Lg, 1u, a.ctr + 3);
    upd_ins_pieces(st, a.run_leaf, a.ctr, m, a.rpieces, a.rsplit, a.pieces);
    launch_scan_u32(st, a.pieces, a.newpos, Lg, a.ctr + 2, a.tmp, a.ctr + 3);
    upd_alloc(st, a.slot_alloc, A_max, a.ctr, ix->free_stack.as<uint32_t>(), dt, cap);
    upd_dir_copy(st, dt, a.ctr, a.pieces, a.newpos, Lg, cap);
    upd_ins_append(st, ix->D, ix->curve, bk, bi, a.run_leaf, a.run_beg, a.ctr, m, a.rsplit, a.newpos, dt,
                   ix->slots.as<uint32_t>(), ix->C, ix->err.as<uint32_t>(), cap);
    if (ix->flags & PSI_FLAG_SORTED_LEAVES) {
        ProfScope ps2(ix, "sort_appended", 0);
        upd_sort_appended(st, ix->D, ix->curve, a.run_leaf, a.ctr, m, a.rsplit, a.newpos, dt,
                          ix->slots.as<uint32_t>(), ix->C, cap);
    }
    upd_ins_split(st, ix->D, ix->curve, NCH_max, bk, bi, a.run_leaf, a.run_beg, a.ctr, m, a.chunk_off, a.piece_off,
                  a.newpos, a.slot_alloc, dt, a.piece_pos, ix->slots.as<uint32_t>(), ix->C, phi, cap);
    upd_piece_meta(st, ix->D, a.piece_pos, A_max, a.ctr, dt, ix->slots.as<uint32_t>(), ix->C, cap);
    upd_ins_free(st, a.run_leaf, a.ctr, m, a.rsplit, a.free_off, dt, ix->free_stack.as<uint32_t>(), cap);
    // an empty index takes the sorted batch as a fresh tree (directory 0,
    // slots from 0); the fill is skipped unless the check chose that
    launch_build_leaves(st, ix->D, ix->curve, bk, bi, m, (m + phi - 1) / phi, ix->C, ix->slots.as<uint32_t>(),
                        ix->pkey[0].as<uint64_t>(), ix->pid[0].as<uint32_t>(), ix->leaf[0].as<NodeRec>(),
                        reinterpret_cast<const uint64_t*>(a.ctr + 12));
    st_ins_commit(st, dt, a.ctr, m, phi, ix->B);
    if ((s = launched()) != PSI_OK) return s;
    if ((s = build_nodes(ix, Lc)) != PSI_OK) return s;
    Bounds d;
    d.L = L_cap - Lb;
    d.slot_top = A_max;
    d.n_free = Fm;
    d.n_live = m;
    d.next_id = m;
    return track_update(ix, d);
}

// Batch delete, queued without waiting, in the same way.
psi_status do_delete(psi_index ix, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted, hipEvent_t before_apply) {
    psi_status s;
    hipStream_t st = ix->st;
    if (m == 0) {
        if (d_ndeleted) launch_fill_u32(st, reinterpret_cast<uint32_t*>(d_ndeleted), 2, 0u);
        return launched();
    }
    Bounds u;
    if ((s = bounds(ix, &u)) != PSI_OK) return s;
    ++ix->gen;
    ProfScope ps(ix, "update", 0);
    const uint32_t phi = ix->phi;
    const uint64_t Lb = u.L;
    // Only leaves the batch touched can fall below the minimum (at most
    // min(L, m)); each regroup takes such leaves plus at most one full
    // neighbour, so at most 2 min(L, m) leaves are freed, the new pieces
    // number at most 3 min(L, m), the directory grows by at most one leaf per
    // group, and the pieces' entries fill at most 2 phi per freed leaf.
    const uint64_t U = std::min(Lb, m);
    const uint64_t A_max = 3 * U + 2;
    const uint64_t F_max = 2 * U + 2;
    const uint64_t L_cap = Lb + U + 2;
    const uint64_t NCH_max = F_max + (2 * (uint64_t)phi * F_max) / UPD_CHUNK + 2;
    if ((s = reserve(ix, u, L_cap, A_max, F_max)) != PSI_OK) return s;
    auto need = [&](uint64_t L) {
        Carver c;
        carve_del(c, m, L, A_max);
        return c.off;
    };
    uint64_t Lg = Lb, Lc = L_cap;
    if ((s = ensure_q(ix, ix->scr.a, need(std::max<uint64_t>(Lb, 1)))) != PSI_OK) return s;
    if ((s = grid_leaves(ix, Lb, L_cap, need, &Lg, &Lc)) != PSI_OK) return s;
    Carver real;
    real.base = static_cast<char*>(ix->scr.a.p);
    DelArrays a = carve_del(real, m, Lg, A_max);
    const Caps cap = caps_of(ix, A_max, Lg, Lc);
    DevTree* dt = ix->dt();
    uint32_t* slots = ix->slots.as<uint32_t>();

    launch_fill_u32(st, a.ctr, 16, 0u);
    st_del_precheck(st, dt, a.ctr, cap);
    // the batch claimed and routed, then grouped by leaf: a sort on the
    // bits of the leaf index only (entries within a leaf need no order)
    int P = 1;
    while (P < 4 && ((1ull << (8 * P)) - 1) < Lg) ++P;
    const uint64_t marker = (1ull << (8 * P)) - 1;  // above every leaf index (< L <= Lg)
    upd_del_take(st, d_ids, m, ix->idkey.as<uint64_t>(), dt, cap.dirs, ix->psample.as<uint4>(), a.ctr, marker, a.dk,
                 a.di);
    int w = 0;
    if ((s = sort_pairs(ix, a.dk, a.di, 0, m, false, false, &w, "radix_update", 0, P)) != PSI_OK) return s;
    a.ci = ix->sorter.i[w].as<uint32_t>();
    upd_del_leaf_of(st, ix->sorter.k[w].as<uint64_t>(), m, a.ctr, a.leaf_of, d_ndeleted);
    upd_runs(st, a.leaf_of, m, a.ctr + 0, a.flag, a.ridx, a.run_leaf, a.run_beg, a.ctr + 1, a.tmp);
    if (before_apply && (s = hip_ok(hipStreamWaitEvent(st, before_apply, 0))) != PSI_OK) return s;
    upd_del_remove(st, ix->D, a.ci, a.run_leaf, a.run_beg, a.ctr, m, dt, slots, ix->C, phi, a.ctr + 8,
                   ix->err.as<uint32_t>(), cap);
    // Leaves below the minimum can only come from this delete (every update
    // leaves all leaves at or above it): with none (ctr[8] = 0) the plan's
    // launches exit at once, F stays 0, and only the node levels change.
    upd_del_plan(st, dt, cap.dirs, Lg, phi, a.ctr, a.cnt, a.cum, a.start, a.gidx, a.grp_first, a.gpieces, a.gchunks, a.galloc,
                 a.gfree, a.gchanged, a.gpos, a.chunk_off, a.alloc_off, a.free_off, a.tmp);
    st_del_check(st, dt, a.ctr, cap);
    upd_alloc(st, a.slot_alloc, A_max, a.ctr, ix->free_stack.as<uint32_t>(), dt, cap);
    upd_del_gcopy(st, a.grp_first, a.ctr, Lg, a.gchanged, a.gpos, dt, cap);
    upd_sort_leaves(st, ix->D, ix->curve, a.start, a.gidx, a.gchanged, a.ctr, Lg, dt, cap.dirs, slots, ix->C);
    upd_del_regroup(st, ix->D, ix->curve, NCH_max, a.grp_first, a.ctr, a.chunk_off, a.alloc_off, a.gpos, a.cum,
                    a.slot_alloc, dt, a.piece_pos, slots, ix->C, phi, cap);
    upd_piece_meta(st, ix->D, a.piece_pos, A_max, a.ctr, dt, slots, ix->C, cap);
    upd_del_free(st, a.start, a.gidx, a.gchanged, a.grp_first, a.free_off, a.ctr, Lg, dt,
                 ix->free_stack.as<uint32_t>(), cap);
    st_del_commit(st, dt, a.ctr, ix->B);
    if ((s = launched()) != PSI_OK) return s;
    if ((s = build_nodes(ix, Lc)) != PSI_OK) return s;
    Bounds d;
    d.L = L_cap - Lb;
    d.slot_top = A_max;
    d.n_free = F_max;
    return track_update(ix, d);
}

}  // namespace psi
