// Launchers of the batch-update kernels (k_update.hip).
#pragma once
#include "psi_kern.h"

namespace psi {

constexpr uint32_t UPD_CHUNK = 256;  // outputs per block when re-cutting leaves

// Sizes of the buffers an update writes through computed indices; kernels
// check every such index against them and latch ERR_CAPACITY instead of
// writing out of bounds.
struct Caps {
    uint64_t leaves;  // entries of the destination directory
    uint64_t slots;   // leaf slots allocated
    uint64_t frees;   // entries of the free-slot stack
    uint64_t alloc;   // slots handed out by this update
    uint32_t* err;    // device error word
};

void upd_route(hipStream_t st, const uint64_t* bk, const uint32_t* bi, uint64_t n, const uint32_t* n_dev,
               const uint64_t* pk, const uint32_t* pi, uint64_t L, uint32_t* leaf_of);
void upd_runs(hipStream_t st, const uint32_t* leaf_of, uint64_t n, const uint32_t* n_dev, uint32_t* flag,
              uint32_t* ridx, uint32_t* run_leaf, uint32_t* run_beg, uint32_t* R_dev, uint32_t* tmp);
void upd_ins_plan(hipStream_t st, const uint32_t* run_leaf, const uint32_t* run_beg, const uint32_t* ctr, uint64_t m,
                  const NodeRec* leaf, uint32_t C, uint32_t phi, uint32_t* rpieces, uint32_t* rchunks,
                  uint32_t* rsplit);
// Re-sorts, by (key, id), every leaf that took a run by appending (leaves in
// total order).
void upd_sort_appended(hipStream_t st, int dim, int curve, const uint32_t* run_leaf, const uint32_t* ctr, uint64_t m,
                       const uint32_t* rsplit, const uint32_t* newpos, const NodeRec* leaf, uint32_t* slots,
                       uint32_t C, Caps cap);
// Piece counts of the re-cut leaves into pieces[] (filled with 1 before).
void upd_ins_pieces(hipStream_t st, const uint32_t* run_leaf, const uint32_t* ctr, uint64_t m, const uint32_t* rpieces,
                    const uint32_t* rsplit, uint32_t* pieces);
void upd_alloc(hipStream_t st, uint32_t* slot_alloc, uint64_t A, const uint32_t* free_stack, uint64_t n_free,
               uint64_t slot_top, Caps cap);
void upd_dir_copy(hipStream_t st, const NodeRec* src, const uint64_t* spk, const uint32_t* spi, const uint32_t* pieces,
                  const uint32_t* newpos, uint64_t L, NodeRec* dst, uint64_t* dpk, uint32_t* dpi, Caps cap);
void upd_ins_append(hipStream_t st, int dim, int curve, const uint64_t* bk, const uint32_t* bi,
                    const uint32_t* run_leaf, const uint32_t* run_beg, const uint32_t* ctr, uint64_t m,
                    const uint32_t* rsplit, const uint32_t* newpos, NodeRec* dleaf, uint64_t* dpk, uint32_t* dpi,
                    uint32_t* slots, uint32_t C, uint32_t* err, Caps cap);
void upd_ins_split(hipStream_t st, int dim, int curve, uint64_t nchunks, const uint64_t* bk, const uint32_t* bi,
                   const uint32_t* run_leaf, const uint32_t* run_beg, const uint32_t* ctr, uint64_t m,
                   const uint32_t* chunk_off, const uint32_t* piece_off, const uint32_t* newpos,
                   const uint32_t* slot_alloc, const NodeRec* sleaf, NodeRec* dleaf, uint64_t* dpk, uint32_t* dpi,
                   uint32_t* piece_pos, uint32_t* slots, uint32_t C, uint32_t phi, Caps cap);
void upd_piece_meta(hipStream_t st, int dim, const uint32_t* piece_pos, uint64_t A, NodeRec* leaf,
                    const uint32_t* slots, uint32_t C, Caps cap);
void upd_ins_free(hipStream_t st, const uint32_t* run_leaf, const uint32_t* ctr, uint64_t m, const uint32_t* rsplit,
                  const uint32_t* free_off, const NodeRec* sleaf, uint32_t* free_stack, uint64_t base, Caps cap);

void upd_del_gather(hipStream_t st, const uint32_t* ids, uint64_t m, const uint64_t* idkey, uint32_t next_id,
                    uint64_t* dk, uint32_t* di);
void upd_del_compact(hipStream_t st, const uint64_t* sk, const uint32_t* si, uint64_t m, uint32_t* flag,
                     uint32_t* pos, uint32_t* V_dev, uint64_t* ck, uint32_t* ci, uint32_t* tmp);
void upd_del_kill(hipStream_t st, const uint32_t* ci, const uint32_t* ctr, uint64_t m, uint64_t* idkey,
                  uint64_t* ndel);
// Removes the runs' ids from their leaves; *under |= 1 if a leaf ends below
// ceil(phi / 2) entries.
void upd_del_remove(hipStream_t st, int dim, const uint32_t* ci, const uint32_t* run_leaf, const uint32_t* run_beg,
                    const uint32_t* ctr, uint64_t m, NodeRec* leaf, uint32_t* slots, uint32_t C, uint32_t phi,
                    uint32_t* under, uint32_t* err, Caps cap);
void upd_del_plan(hipStream_t st, const NodeRec* leaf, uint64_t L, uint32_t phi, uint32_t* ctr, uint32_t* cnt,
                  uint32_t* cum, uint32_t* start, uint32_t* gidx, uint32_t* grp_first, uint32_t* gpieces,
                  uint32_t* gchunks, uint32_t* galloc, uint32_t* gfree, uint32_t* gchanged, uint32_t* gpos,
                  uint32_t* chunk_off, uint32_t* alloc_off, uint32_t* free_off, uint32_t* tmp);
void upd_del_gcopy(hipStream_t st, const uint32_t* grp_first, const uint32_t* ctr, uint64_t L,
                   const uint32_t* gchanged, const uint32_t* gpos, const NodeRec* src, const uint64_t* spk,
                   const uint32_t* spi, NodeRec* dst, uint64_t* dpk, uint32_t* dpi, Caps cap);
void upd_sort_leaves(hipStream_t st, int dim, int curve, const uint32_t* start, const uint32_t* gidx,
                     const uint32_t* gchanged, uint64_t L, const NodeRec* leaf, uint32_t* slots, uint32_t C);
void upd_del_regroup(hipStream_t st, int dim, int curve, uint64_t nchunks, const uint32_t* grp_first,
                     const uint32_t* ctr, uint64_t L, const uint32_t* chunk_off, const uint32_t* alloc_off,
                     const uint32_t* gpos, const uint32_t* cum, const uint32_t* slot_alloc, const NodeRec* sleaf,
                     NodeRec* dleaf, uint64_t* dpk, uint32_t* dpi, uint32_t* piece_pos, uint32_t* slots, uint32_t C,
                     uint32_t phi, Caps cap);
void upd_del_free(hipStream_t st, const uint32_t* start, const uint32_t* gidx, const uint32_t* gchanged,
                  const uint32_t* grp_first, const uint32_t* free_off, uint64_t L, const NodeRec* sleaf,
                  uint32_t* free_stack, uint64_t base, Caps cap);

}  // namespace psi
