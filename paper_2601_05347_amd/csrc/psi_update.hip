// Batch insert (Alg. 4) and batch delete (Sec. 4.2): host orchestration.
//
// Both calls sort the batch's (key, id) pairs, route them to leaves, change
// the touched leaves, and only then learn (one wait on the stream) how many
// leaves and slots the new directory needs. When no leaf is re-cut the
// directory is updated in place; otherwise a new directory is written into
// the inactive buffer: untouched leaves are copied, re-cut leaves get fresh
// slots, and the freed slots go to a free stack reused by later updates.
// Node levels are rebuilt over the new directory at the end.
#include <algorithm>
#include <cstring>

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

// Slot storage for `need_new` more slots and a free stack of `cap` entries.
psi_status reserve_slots(psi_index ix, uint64_t A, uint64_t F, uint64_t* new_top, uint64_t* n_free_after,
                         uint64_t* push_base) {
    const uint64_t take_free = std::min<uint64_t>(A, ix->n_free);
    *new_top = ix->slot_top + (A - take_free);
    *push_base = ix->n_free - take_free;
    *n_free_after = *push_base + F;
    const uint64_t sw = ix->slot_words() * 4;
    psi_status s = ix->slots.grow_keep(*new_top * sw, ix->slot_top * sw, ix->st);
    if (s != PSI_OK) return s;
    return ix->free_stack.grow_keep(std::max(*n_free_after, ix->n_free) * 4 + 4, ix->n_free * 4, ix->st);
}

Caps caps_of(psi_index ix, int dst, uint64_t A) {
    Caps c;
    c.leaves = std::min(ix->leaf[dst].bytes / sizeof(NodeRec),
                        std::min(ix->pkey[dst].bytes / 8, ix->pid[dst].bytes / 4));
    c.slots = ix->slots.bytes / (ix->slot_words() * 4);
    c.frees = ix->free_stack.bytes / 4;
    c.alloc = A;
    c.err = ix->err.as<uint32_t>();
    return c;
}

psi_status ensure_dir(psi_index ix, int which, uint64_t L) {
    psi_status s;
    if ((s = ix->leaf[which].ensure(std::max<uint64_t>(L, 1) * sizeof(NodeRec))) != PSI_OK) return s;
    if ((s = ix->pkey[which].ensure(std::max<uint64_t>(L, 1) * 8)) != PSI_OK) return s;
    return ix->pid[which].ensure(std::max<uint64_t>(L, 1) * 4);
}

}  // namespace

psi_status do_insert(psi_index ix, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids) {
    psi_status s;
    hipStream_t st = ix->st;
    const uint32_t base_id = ix->next_id;
    if (ix->L == 0) {  // empty index: a build whose ids continue from next_id
        if ((s = do_build(ix, d_pts, m, base_id)) != PSI_OK) return s;
        if (d_new_ids) launch_iota_u32(st, d_new_ids, m, base_id);
        ix->next_id = base_id + (uint32_t)m;
        return launched();
    }
    ProfScope ps(ix, "update", 0);
    if ((s = ix->idkey.grow_keep(((uint64_t)base_id + m) * 8, (uint64_t)base_id * 8, st)) != PSI_OK) return s;
    Sorter& S = ix->sorter;
    if ((s = S.hist.ensure(MAX_PASSES * RADIX * 4)) != PSI_OK) return s;
    launch_fill_u32(st, S.hist.as<uint32_t>(), 8 * RADIX, 0u);
    uint64_t* keys = ix->idkey.as<uint64_t>() + base_id;
    launch_encode_hist(st, ix->D, ix->curve, d_pts, m, keys, S.hist.as<uint32_t>(), ix->err.as<uint32_t>());
    int w = 0;
    if ((s = sort_pairs(ix, keys, nullptr, base_id, m, false, true, &w, "radix_update")) != PSI_OK) return s;
    const uint64_t* bk = S.k[w].as<uint64_t>();
    const uint32_t* bi = S.i[w].as<uint32_t>();
    if (d_new_ids) launch_iota_u32(st, d_new_ids, m, base_id);

    const uint64_t L = ix->L;
    const int cur = ix->cur;
    Carver cv;
    auto carve = [&](Carver& c) {
        struct {
            uint32_t *ctr, *leaf_of, *flag, *ridx, *run_leaf, *run_beg, *rpieces, *rchunks, *rsplit, *piece_off,
                *chunk_off, *free_off, *pieces, *newpos, *tmp;
        } a;
        a.ctr = c.take<uint32_t>(16);
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
        return a;
    };
    carve(cv);
    if ((s = ix->scr.a.ensure(cv.off)) != PSI_OK) return s;
    Carver real;
    real.base = static_cast<char*>(ix->scr.a.p);
    auto a = carve(real);

    launch_fill_u32(st, a.ctr, 16, 0u);
    upd_route(st, bk, bi, m, nullptr, ix->pkey[cur].as<uint64_t>(), ix->pid[cur].as<uint32_t>(), L, a.leaf_of);
    upd_runs(st, a.leaf_of, m, nullptr, a.flag, a.ridx, a.run_leaf, a.run_beg, a.ctr + 1, a.tmp);
    upd_ins_plan(st, a.run_leaf, a.run_beg, a.ctr, m, ix->leaf[cur].as<NodeRec>(), ix->C, ix->phi, a.rpieces,
                 a.rchunks, a.rsplit);
    ScanSet sc{{a.rpieces, a.rchunks, a.rsplit, nullptr},
               {a.piece_off, a.chunk_off, a.free_off, nullptr},
               {a.ctr + 3, a.ctr + 4, a.ctr + 5, nullptr},
               {m, m, m, 0}};
    launch_scan_multi(st, sc, 3, a.tmp);
    if ((s = launched()) != PSI_OK) return s;
    if ((s = readback(ix, a.ctr, 8 * 4)) != PSI_OK) return s;
    uint32_t c[8];
    std::memcpy(c, ix->pinned, sizeof c);
    // A new slots (pieces of the re-cut leaves), F re-cut leaves (one freed
    // slot each): L - F + A leaves after the splice
    const uint64_t A = c[3], NCH = c[4], F = c[5];
    if (F > L || F > A) return PSI_E_INTERNAL;
    const uint64_t Lnew = L - F + A;

    const bool recut = A > 0;
    if (recut) {  // new directory positions: exclusive scan of the per-leaf piece counts
        launch_fill_u32(st, a.pieces, L, 1u);
        upd_ins_pieces(st, a.run_leaf, a.ctr, m, a.rpieces, a.rsplit, a.pieces);
        launch_scan_u32(st, a.pieces, a.newpos, L, a.ctr + 2, a.tmp);
    }
    const int dst = recut ? 1 - cur : cur;
    if (recut && (s = ensure_dir(ix, dst, Lnew)) != PSI_OK) return s;
    uint64_t new_top = ix->slot_top, n_free_after = ix->n_free, push_base = ix->n_free;
    if ((s = reserve_slots(ix, A, F, &new_top, &n_free_after, &push_base)) != PSI_OK) return s;
    if ((s = ix->scr.b.ensure(2 * ((A + 1) * 4 + 256))) != PSI_OK) return s;
    Carver cb;
    cb.base = static_cast<char*>(ix->scr.b.p);
    uint32_t* slot_alloc = cb.take<uint32_t>(A);
    uint32_t* piece_pos = cb.take<uint32_t>(A);
    const Caps cap = caps_of(ix, dst, A);
    upd_alloc(st, slot_alloc, A, ix->free_stack.as<uint32_t>(), ix->n_free, ix->slot_top, cap);
    NodeRec* dleaf = ix->leaf[dst].as<NodeRec>();
    uint64_t* dpk = ix->pkey[dst].as<uint64_t>();
    uint32_t* dpi = ix->pid[dst].as<uint32_t>();
    if (recut)
        upd_dir_copy(st, ix->leaf[cur].as<NodeRec>(), ix->pkey[cur].as<uint64_t>(), ix->pid[cur].as<uint32_t>(),
                     a.pieces, a.newpos, L, dleaf, dpk, dpi, cap);
    upd_ins_append(st, ix->D, ix->curve, bk, bi, a.run_leaf, a.run_beg, a.ctr, m, a.rsplit,
                   recut ? a.newpos : nullptr, dleaf, dpk, dpi, ix->slots.as<uint32_t>(), ix->C,
                   ix->err.as<uint32_t>(), cap);
    if (ix->flags & PSI_FLAG_SORTED_LEAVES) {
        ProfScope ps(ix, "sort_appended", 0);
        upd_sort_appended(st, ix->D, ix->curve, a.run_leaf, a.ctr, m, a.rsplit, recut ? a.newpos : nullptr, dleaf,
                          ix->slots.as<uint32_t>(), ix->C, cap);
    }
    if (recut) {
        upd_ins_split(st, ix->D, ix->curve, NCH, bk, bi, a.run_leaf, a.run_beg, a.ctr, m, a.chunk_off, a.piece_off,
                      a.newpos, slot_alloc, ix->leaf[cur].as<NodeRec>(), dleaf, dpk, dpi, piece_pos,
                      ix->slots.as<uint32_t>(), ix->C, ix->phi, cap);
        upd_piece_meta(st, ix->D, piece_pos, A, dleaf, ix->slots.as<uint32_t>(), ix->C, cap);
        upd_ins_free(st, a.run_leaf, a.ctr, m, a.rsplit, a.free_off, ix->leaf[cur].as<NodeRec>(),
                     ix->free_stack.as<uint32_t>(), push_base, cap);
        ix->cur = dst;
    }
    if ((s = launched()) != PSI_OK) return s;
    ix->slot_top = new_top;
    ix->n_free = n_free_after;
    ix->L = Lnew;
    ix->n_live += m;
    ix->next_id = base_id + (uint32_t)m;
    return build_nodes(ix);
}

psi_status do_delete(psi_index ix, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted) {
    psi_status s;
    hipStream_t st = ix->st;
    if (m == 0 || ix->L == 0) {
        if (d_ndeleted) launch_fill_u32(st, reinterpret_cast<uint32_t*>(d_ndeleted), 2, 0u);
        return launched();
    }
    ProfScope ps(ix, "update", 0);
    const uint64_t L = ix->L;
    const int cur = ix->cur;
    auto carve = [&](Carver& c) {
        struct {
            uint32_t* ctr;
            uint64_t *dk, *ck;
            uint32_t *di, *flag, *pos, *ci, *leaf_of, *ridx, *run_leaf, *run_beg;
            uint32_t *cnt, *cum, *start, *gidx, *grp_first, *gpieces, *gchunks, *galloc, *gfree, *gchanged, *gpos,
                *chunk_off, *alloc_off, *free_off, *tmp;
        } a;
        a.ctr = c.take<uint32_t>(16);
        a.dk = c.take<uint64_t>(m);
        a.ck = c.take<uint64_t>(m);
        a.di = c.take<uint32_t>(m);
        a.flag = c.take<uint32_t>(m);
        a.pos = c.take<uint32_t>(m);
        a.ci = c.take<uint32_t>(m);
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
        return a;
    };
    Carver cv;
    carve(cv);
    if ((s = ix->scr.a.ensure(cv.off)) != PSI_OK) return s;
    Carver real;
    real.base = static_cast<char*>(ix->scr.a.p);
    auto a = carve(real);

    launch_fill_u32(st, a.ctr, 16, 0u);
    upd_del_gather(st, d_ids, m, ix->idkey.as<uint64_t>(), ix->next_id, a.dk, a.di);
    int w = 0;
    if ((s = sort_pairs(ix, a.dk, a.di, 0, m, true, false, &w, "radix_update")) != PSI_OK) return s;
    upd_del_compact(st, ix->sorter.k[w].as<uint64_t>(), ix->sorter.i[w].as<uint32_t>(), m, a.flag, a.pos, a.ctr + 0,
                    a.ck, a.ci, a.tmp);
    upd_del_kill(st, a.ci, a.ctr, m, ix->idkey.as<uint64_t>(), d_ndeleted);
    upd_route(st, a.ck, a.ci, m, a.ctr + 0, ix->pkey[cur].as<uint64_t>(), ix->pid[cur].as<uint32_t>(), L, a.leaf_of);
    upd_runs(st, a.leaf_of, m, a.ctr + 0, a.flag, a.ridx, a.run_leaf, a.run_beg, a.ctr + 1, a.tmp);
    upd_del_remove(st, ix->D, a.ci, a.run_leaf, a.run_beg, a.ctr, m, ix->leaf[cur].as<NodeRec>(),
                   ix->slots.as<uint32_t>(), ix->C, ix->phi, a.ctr + 8, ix->err.as<uint32_t>(), caps_of(ix, cur, 0));
    // Leaves below the minimum can only come from this delete (every update
    // leaves all leaves at or above it): with none (ctr[8] = 0) the plan's
    // launches exit at once, F stays 0, and only the node levels change.
    upd_del_plan(st, ix->leaf[cur].as<NodeRec>(), L, ix->phi, a.ctr, a.cnt, a.cum, a.start, a.gidx, a.grp_first,
                 a.gpieces, a.gchunks, a.galloc, a.gfree, a.gchanged, a.gpos, a.chunk_off, a.alloc_off, a.free_off,
                 a.tmp);
    if ((s = launched()) != PSI_OK) return s;
    if ((s = readback(ix, a.ctr, 8 * 4)) != PSI_OK) return s;
    uint32_t c[8];
    std::memcpy(c, ix->pinned, sizeof c);
    const uint64_t V = c[0], Lnew = c[2], A = c[3], NCH = c[4], F = c[5];
    ix->n_live -= std::min<uint64_t>(V, ix->n_live);
    if (F > 0) {
        const int dst = 1 - cur;
        if ((s = ensure_dir(ix, dst, Lnew)) != PSI_OK) return s;
        uint64_t new_top, n_free_after, push_base;
        if ((s = reserve_slots(ix, A, F, &new_top, &n_free_after, &push_base)) != PSI_OK) return s;
        if ((s = ix->scr.b.ensure(2 * ((A + 1) * 4 + 256))) != PSI_OK) return s;
        Carver cb;
        cb.base = static_cast<char*>(ix->scr.b.p);
        uint32_t* slot_alloc = cb.take<uint32_t>(A);
        uint32_t* piece_pos = cb.take<uint32_t>(A);
        NodeRec* sleaf = ix->leaf[cur].as<NodeRec>();
        NodeRec* dleaf = ix->leaf[dst].as<NodeRec>();
        uint64_t* dpk = ix->pkey[dst].as<uint64_t>();
        uint32_t* dpi = ix->pid[dst].as<uint32_t>();
        uint32_t* slots = ix->slots.as<uint32_t>();
        const Caps cap = caps_of(ix, dst, A);
        upd_alloc(st, slot_alloc, A, ix->free_stack.as<uint32_t>(), ix->n_free, ix->slot_top, cap);
        upd_del_gcopy(st, a.grp_first, a.ctr, L, a.gchanged, a.gpos, sleaf, ix->pkey[cur].as<uint64_t>(),
                      ix->pid[cur].as<uint32_t>(), dleaf, dpk, dpi, cap);
        upd_sort_leaves(st, ix->D, ix->curve, a.start, a.gidx, a.gchanged, L, sleaf, slots, ix->C);
        upd_del_regroup(st, ix->D, ix->curve, NCH, a.grp_first, a.ctr, L, a.chunk_off, a.alloc_off, a.gpos, a.cum,
                        slot_alloc, sleaf, dleaf, dpk, dpi, piece_pos, slots, ix->C, ix->phi, cap);
        upd_piece_meta(st, ix->D, piece_pos, A, dleaf, slots, ix->C, cap);
        upd_del_free(st, a.start, a.gidx, a.gchanged, a.grp_first, a.free_off, L, sleaf,
                     ix->free_stack.as<uint32_t>(), push_base, cap);
        if ((s = launched()) != PSI_OK) return s;
        ix->cur = dst;
        ix->slot_top = new_top;
        ix->n_free = n_free_after;
        ix->L = Lnew;
    }
    return build_nodes(ix);
}

}  // namespace psi
