// Launchers of the batch-update kernels (k_update.hip).
#pragma once
#include "psi_kern.h"

namespace psi {

constexpr uint32_t UPD_CHUNK = 256;  // outputs per block when re-cutting leaves

// Sizes of the buffers an update writes through computed indices; kernels
// check every such index against them and latch ERR_CAPACITY instead of
// writing out of bounds.
// lgrid: leaves the update's per-leaf grids and arrays cover (an update
// finding more leaves than that is refused before it changes anything).
struct Caps {
    uint64_t leaves;  // entries of the destination directory (and leaves the node grids cover)
    uint64_t slots;   // leaf slots allocated
    uint64_t frees;   // entries of the free-slot stack
    uint64_t alloc;   // slots handed out by this update
    uint64_t lgrid;   // leaves the per-leaf grids cover
    uint32_t* err;    // device error word
    Dirs dirs;        // the directory buffers
};

void upd_route(hipStream_t st, const uint64_t* bk, const uint32_t* bi, uint64_t n, const uint32_t* n_dev,
               const DevTree* dt, const Dirs& dirs, uint32_t* leaf_of);
void upd_runs(hipStream_t st, const uint32_t* leaf_of, uint64_t n, const uint32_t* n_dev, uint32_t* flag,
              uint32_t* ridx, uint32_t* run_leaf, uint32_t* run_beg, uint32_t* R_dev, uint32_t* tmp);
void upd_ins_plan(hipStream_t st, const uint32_t* run_leaf, const uint32_t* run_beg, const uint32_t* ctr, uint64_t m,
                  const DevTree* dt, const Dirs& dirs, uint32_t phi, uint32_t* rpieces, uint32_t* rchunks,
                  uint32_t* rsplit);
// Re-sorts, by (key, id), every leaf that took a run by appending (leaves in
// total order).
void upd_sort_appended(hipStream_t st, int dim, int curve, const uint32_t* run_leaf, const uint32_t* ctr, uint64_t m,
                       const uint32_t* rsplit, const uint32_t* newpos, const DevTree* dt, uint32_t* slots,
                       uint32_t C, Caps cap);
// Piece counts of the re-cut leaves into pieces[] (filled with 1 before).
void upd_ins_pieces(hipStream_t st, const uint32_t* run_leaf, const uint32_t* ctr, uint64_t m, const uint32_t* rpieces,
                    const uint32_t* rsplit, uint32_t* pieces);
// Slots for the ctr[3] new leaves (A_max bounds ctr[3]: the grid).
void upd_alloc(hipStream_t st, uint32_t* slot_alloc, uint64_t A_max, const uint32_t* ctr, const uint32_t* free_stack,
               const DevTree* dt, Caps cap);
void upd_dir_copy(hipStream_t st, const DevTree* dt, const uint32_t* ctr, const uint32_t* pieces,
                  const uint32_t* newpos, uint64_t Lb, Caps cap);
void upd_ins_append(hipStream_t st, int dim, int curve, const uint64_t* bk, const uint32_t* bi,
                    const uint32_t* run_leaf, const uint32_t* run_beg, const uint32_t* ctr, uint64_t m,
                    const uint32_t* rsplit, const uint32_t* newpos, const DevTree* dt, uint32_t* slots, uint32_t C,
                    uint32_t* err, Caps cap);
void upd_ins_split(hipStream_t st, int dim, int curve, uint64_t nch_max, const uint64_t* bk, const uint32_t* bi,
                   const uint32_t* run_leaf, const uint32_t* run_beg, const uint32_t* ctr, uint64_t m,
                   const uint32_t* chunk_off, const uint32_t* piece_off, const uint32_t* newpos,
                   const uint32_t* slot_alloc, const DevTree* dt, uint32_t* piece_pos, uint32_t* slots, uint32_t C,
                   uint32_t phi, Caps cap);
void upd_piece_meta(hipStream_t st, int dim, const uint32_t* piece_pos, uint64_t A_max, const uint32_t* ctr,
                    const DevTree* dt, const uint32_t* slots, uint32_t C, Caps cap);
void upd_ins_free(hipStream_t st, const uint32_t* run_leaf, const uint32_t* ctr, uint64_t m, const uint32_t* rsplit,
                  const uint32_t* free_off, const DevTree* dt, uint32_t* free_stack, Caps cap);

// Claims the batch's live ids (their keys in idkey become the dead mark),
// routes them to their leaves and writes the sort keys (leaf index, or
// `marker` for a dropped id) and ids; ctr[0] += the number claimed.
// samp: the pivot sample of the current directory (first routing steps).
void upd_del_take(hipStream_t st, const uint32_t* ids, uint64_t m, uint64_t* idkey, const DevTree* dt, const Dirs& dirs,
                  const uint4* samp, uint32_t* ctr, uint64_t marker, uint64_t* lk, uint32_t* li);
// leaf_of[e] = low word of the sorted key e; *ndel (nullable) = ctr[0].
void upd_del_leaf_of(hipStream_t st, const uint64_t* sk, uint64_t m, const uint32_t* ctr, uint32_t* leaf_of,
                     uint64_t* ndel);
// Removes the runs' ids from their leaves; *under |= 1 if a leaf ends below
// ceil(phi / 2) entries.
void upd_del_remove(hipStream_t st, int dim, const uint32_t* ci, const uint32_t* run_leaf, const uint32_t* run_beg,
                    const uint32_t* ctr, uint64_t m, const DevTree* dt, uint32_t* slots, uint32_t C, uint32_t phi,
                    uint32_t* under, uint32_t* err, Caps cap);
// Regrouping plan over the Lb >= L entries of the per-leaf arrays.
void upd_del_plan(hipStream_t st, const DevTree* dt, const Dirs& dirs, uint64_t Lb, uint32_t phi, uint32_t* ctr, uint32_t* cnt,
                  uint32_t* cum, uint32_t* start, uint32_t* gidx, uint32_t* grp_first, uint32_t* gpieces,
                  uint32_t* gchunks, uint32_t* galloc, uint32_t* gfree, uint32_t* gchanged, uint32_t* gpos,
                  uint32_t* chunk_off, uint32_t* alloc_off, uint32_t* free_off, uint32_t* tmp);
void upd_del_gcopy(hipStream_t st, const uint32_t* grp_first, const uint32_t* ctr, uint64_t Lb,
                   const uint32_t* gchanged, const uint32_t* gpos, const DevTree* dt, Caps cap);
void upd_sort_leaves(hipStream_t st, int dim, int curve, const uint32_t* start, const uint32_t* gidx,
                     const uint32_t* gchanged, const uint32_t* ctr, uint64_t Lb, const DevTree* dt, const Dirs& dirs,
                     uint32_t* slots, uint32_t C);
void upd_del_regroup(hipStream_t st, int dim, int curve, uint64_t nch_max, const uint32_t* grp_first,
                     const uint32_t* ctr, const uint32_t* chunk_off, const uint32_t* alloc_off,
                     const uint32_t* gpos, const uint32_t* cum, const uint32_t* slot_alloc, const DevTree* dt,
                     uint32_t* piece_pos, uint32_t* slots, uint32_t C, uint32_t phi, Caps cap);
void upd_del_free(hipStream_t st, const uint32_t* start, const uint32_t* gidx, const uint32_t* gchanged,
                  const uint32_t* grp_first, const uint32_t* free_off, const uint32_t* ctr, uint64_t Lb,
                  const DevTree* dt, uint32_t* free_stack, Caps cap);

// Device state (k_state.hip).
void st_set_dirs(hipStream_t st, DevTree* dt, NodeRec* l0, NodeRec* l1, uint64_t* k0, uint64_t* k1, uint32_t* i0,
                 uint32_t* i1);
void st_reset(hipStream_t st, DevTree* dt, uint32_t B);
void st_commit_build(hipStream_t st, DevTree* dt, uint64_t n, uint64_t L, uint32_t cur, uint32_t next_id,
                     uint32_t B);
void st_ins_ids(hipStream_t st, const DevTree* dt, const uint64_t* keys, uint64_t m, uint64_t* idkey, uint64_t id_cap,
                uint32_t* bi, uint32_t* new_ids, const uint32_t* ctr);
void st_ins_check(hipStream_t st, const DevTree* dt, uint32_t* ctr, uint64_t m, uint32_t phi, uint64_t id_cap,
                  Caps cap);
void st_ins_commit(hipStream_t st, DevTree* dt, const uint32_t* ctr, uint64_t m, uint32_t phi, uint32_t B);
void st_del_check(hipStream_t st, const DevTree* dt, uint32_t* ctr, Caps cap);
// Before a delete removes anything: more leaves than its grids cover makes
// it remove nothing (ctr[0] = 0) and latch ERR_CAPACITY.
void st_del_precheck(hipStream_t st, const DevTree* dt, uint32_t* ctr, Caps cap);
void st_del_commit(hipStream_t st, DevTree* dt, const uint32_t* ctr, uint32_t B);
void st_fill_gated(hipStream_t st, uint32_t* p, uint64_t n, uint32_t v, const uint32_t* gate);

}  // namespace psi
