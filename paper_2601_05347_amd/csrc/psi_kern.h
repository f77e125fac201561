// Host-callable launchers of the gfx950 kernels (one translation unit per
// kernel family). All launches are asynchronous on the given stream.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stddef.h>

#include "psi_dev.h"

namespace psi {

// The two directory buffers, passed to kernels by value: pointers that come
// in as kernel arguments are known to address device memory (global loads),
// while pointers read from memory would be loaded through the slower flat
// path. DevTree::cur says which one is current.
struct Dirs {
    NodeRec* leaf[2];
    uint64_t* pkey[2];
    uint32_t* pid[2];
};

// The mutable state of one index, kept in device memory so that updates are
// planned, applied and committed by kernels alone (the host never has to read
// a count back to size the next launch). Kernels read the leaf count, the
// current directory buffer and the node layout from here; the host sizes its
// launches and buffers by upper bounds of these values.
struct DevTree {
    NodeRec* leaf[2];    // the two directory buffers; leaf[cur] is current
    uint64_t* pkey[2];   // pivot keys, same buffers
    uint32_t* pid[2];    // pivot ids
    uint64_t L;          // leaves in the current directory
    uint64_t n_inner;    // inner nodes (levels 0 .. h-1)
    uint64_t n_live;     // live points
    uint64_t slot_top;   // leaf slots ever handed out (bump pointer)
    uint64_t n_free;     // entries of the free-slot stack
    uint32_t cur;        // current directory buffer
    uint32_t h;          // height: levels 0 .. h, level h = the leaves
    uint32_t next_id;    // next id an insert hands out
    uint32_t sort_top;   // bucket bits of the last two-level build sort (~0: none yet)
    LevelInfo lv[MAX_LEVELS];  // levels 0 .. h
};
// Bytes of the DevTree head (everything before the level table): what the
// host mirrors after each update to tighten its upper bounds.
constexpr size_t DEVTREE_HEAD = offsetof(DevTree, lv);

// ------------------------------------------------------------- radix sort
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 256;
constexpr int SORT_WG = 256;
constexpr int SORT_IPT = 16;
constexpr int SORT_TILE = SORT_WG * SORT_IPT;  // 4096 pairs per tile
constexpr int MAX_PASSES = 12;

// One LSD pass: which word supplies the digit (0 = key, 1 = id) and where.
struct PassList {
    int n;
    uint8_t src[MAX_PASSES];
    uint8_t shift[MAX_PASSES];
};

// Up to SORT_SMALL_MAX pairs: all passes of pl (src 0: key byte at shift,
// 1: id byte) in one launch of one workgroup; stable, like the global passes.
// iin == nullptr: id = id_base + position.
constexpr uint32_t SORT_SMALL_MAX = 10240;
void launch_sort_small(hipStream_t st, const uint64_t* kin, const uint32_t* iin, uint32_t id_base, uint32_t n,
                       const PassList& pl, uint64_t* kout, uint32_t* iout);

// Histograms of every pass's digit over the input pairs; ids == nullptr means
// id = id_base + position. hist must be zeroed ([pl.n][256] u32).
void launch_hist_pairs(hipStream_t st, const uint64_t* keys, const uint32_t* ids, uint32_t id_base,
                       uint64_t n, const PassList& pl, uint32_t* hist);
// Curve keys of points (AoS) -> keys[i]; histograms of `rows` 8-bit key
// digits (row r: bits shift0 + 8 r ..; hist zeroed, [rows][256], rows <= 8);
// coordinates out of range set ERR_RANGE.
void launch_encode_hist(hipStream_t st, int dim, int curve, const uint32_t* pts, uint64_t n, uint64_t* keys,
                        uint32_t* hist, uint32_t* err, int rows = 8, uint32_t shift0 = 0);
// Curve keys of box centres (boxes [n][2][dim]); used to order box batches.
void launch_encode_boxes(hipStream_t st, int dim, int curve, const uint32_t* boxes, uint64_t n, uint64_t* keys);
// Curve keys only; kmax (optional, zeroed by the caller) receives the
// largest key.
void launch_encode(hipStream_t st, int dim, int curve, const uint32_t* pts, uint64_t n, uint64_t* keys,
                   uint32_t* err, uint64_t* kmax = nullptr);
// Curve keys, the largest key (kmax, zeroed by the caller) and the
// per-chunk bucket digit counts for bucket bits [s0, s0 + 16), as
// launch_hist_chunks makes them (cnt [2][XCD_CHUNKS][256], zeroed).
void launch_encode_chunks(hipStream_t st, int dim, int curve, const uint32_t* pts, uint64_t n, uint64_t* keys,
                          uint32_t* err, uint64_t* kmax, uint32_t s0, uint32_t* cnt);
// Exclusive scan of every pass's 256 counts: off[p][d].
void launch_digit_offsets(hipStream_t st, int npass, const uint32_t* hist, uint32_t* off);
// One stable scatter pass (decoupled look-back over tiles taken in launch
// order). status holds n_tiles*256 words tagged with `epoch`; tile_ctr must
// be zero.
// Segmented sorts (many independent indexes in one launch): tile t covers
// [tile_beg[t], min(tile_beg[t] + SORT_TILE, seg_end[tile_seg[t]])); digit
// offsets are per segment at dig_off + seg * off_stride.
struct SegTiles {
    const uint32_t* tile_seg;
    const uint32_t* tile_beg;
    const uint32_t* seg_first_tile;
    const uint32_t* seg_end;
    uint32_t off_stride;
};
// A pass cut into XCD_CHUNKS chunks of consecutive tiles, one per XCD (the
// workgroups with blockIdx % XCD_CHUNKS == x sort chunk x); device arrays of
// XCD_CHUNKS entries. Tiles of chunk x: global tile ids first_tile[x] ..
// first_tile[x] + ntiles[x] - 1 covering positions [pos_begin[x], pos_end[x]).
constexpr uint32_t XCD_CHUNKS = 8;
struct XcdChunks {
    const uint32_t* first_tile;
    const uint32_t* ntiles;
    const uint64_t* pos_begin;
    const uint64_t* pos_end;
};
// A segmented pass with ntiles_dev (device word, may be null) takes tiles
// while fewer than *ntiles_dev are taken, with seg_tiles workgroups that
// each take as many as they can (else one workgroup per tile).
void launch_onesweep(hipStream_t st, bool implicit_ids, bool digit_from_id, const uint64_t* kin,
                     const uint32_t* iin, uint32_t id_base, uint64_t* kout, uint32_t* iout, uint64_t n,
                     uint32_t shift, const uint32_t* dig_off, uint64_t* status, uint32_t* tile_ctr,
                     uint32_t epoch, uint32_t* err, const SegTiles* seg = nullptr, uint64_t seg_tiles = 0,
                     const uint32_t* ntiles_dev = nullptr);
// Chunked pass: dig_off is [XCD_CHUNKS][256] (chunk x's destination of digit
// d); tile_ctr holds XCD_CHUNKS zeroed counters; XCD_CHUNKS * wg_per_chunk
// workgroups take one tile each; with `overflow`, a second small launch
// takes whatever tiles are left (chunks of data-dependent sizes: any
// wg_per_chunk >= 1 is then correct); without it wg_per_chunk must bound
// every chunk's tiles. The digit sits at bit shift (+ *shift_dev if
// shift_dev is not null).
void launch_onesweep_xcd(hipStream_t st, bool implicit_ids, const uint64_t* kin, const uint32_t* iin,
                         uint32_t id_base, uint64_t* kout, uint32_t* iout, uint64_t n, uint32_t shift,
                         const uint32_t* dig_off, uint64_t* status, uint32_t* tile_ctr, uint32_t epoch, uint32_t* err,
                         const XcdChunks& xc, uint32_t wg_per_chunk, const uint32_t* shift_dev = nullptr,
                         bool overflow = false);
void launch_fill_u32(hipStream_t st, uint32_t* p, uint64_t n, uint32_t v);
void launch_iota_u32(hipStream_t st, uint32_t* p, uint64_t n, uint32_t base);

// ------------------------------------------------- two-level build sort
// Pairs already ordered by their top bits (key >> shift) fall into buckets;
// a bucket of at most BUCKET_MAX pairs is sorted in one workgroup's LDS.
// Buckets are the 16 key bits [top, top + 16) just below the largest key's
// leading bit.
constexpr int BUCKET_MAX = 4096;
constexpr int BUCKET_SMALL = 2048;  // lighter variant (half the LDS) for the common bucket sizes
constexpr int BUCKET_HUGE = 8192;   // 1024-thread variant (112 KB of LDS) for BUCKET_MAX + 1 .. BUCKET_HUGE
constexpr uint32_t BUCKET_COUNT = 1u << 16;
// Histograms of two 8-bit key digits (rows at bits s0 and s1; hist [2][256],
// zeroed).
void launch_hist_keys2(hipStream_t st, const uint64_t* keys, uint64_t n, uint32_t s0, uint32_t s1, uint32_t* hist);
// Chunked bucket passes: cnt ([2][XCD_CHUNKS][256], zeroed) counts the first
// digit per input chunk and the second digit per group of 32 first-digit
// values; launch_chunk_offsets turns them into per-chunk digit offsets
// (off1, off2: [XCD_CHUNKS][256]) and the chunk tables of both passes.
struct ChunkTables {
    uint32_t* first_tile;
    uint32_t* ntiles;
    uint64_t* pos_begin;
    uint64_t* pos_end;
};
// With redo (device word, may be null): counts only if *redo != 0, on the
// digits at bits *top and *top + 8.
void launch_hist_chunks(hipStream_t st, const uint64_t* keys, uint64_t n, uint32_t s0, uint32_t s1, uint32_t* cnt,
                        const uint32_t* redo = nullptr, const uint32_t* top = nullptr);
// *top = bucket bits of the largest key *kmax (16 below its leading bit);
// *redo = (*top != guess).
void launch_fix_top(hipStream_t st, const uint64_t* kmax, uint32_t guess, uint32_t* top, uint32_t* redo);
// Zeroes words_per * (*count) words (count <= max_count).
void launch_zero_counted(hipStream_t st, uint32_t* p, uint64_t words_per, const uint32_t* count, uint64_t max_count);
void launch_chunk_offsets(hipStream_t st, const uint32_t* cnt, uint64_t n, uint32_t* off1, uint32_t* off2,
                          ChunkTables tb1, ChunkTables tb2);
// bstart[t] for t in [0, nb] (nb + 1 words): first position of bucket t.
// The bucket bits start at bit *top (device word).
void launch_bucket_starts(hipStream_t st, const uint64_t* keys, uint64_t n, const uint32_t* top, uint32_t* bstart,
                          uint32_t nb);
// Sorts buckets by (key, id) in place, in two launches: wide = false takes
// every bucket of at most BUCKET_SMALL pairs and sets big[t] = 1 for the
// larger ones (2 for a skewed one it leaves alone, else 0); wide = true then
// takes those of at most BUCKET_MAX and the skewed ones and clears their
// flag. Decreasing bucket starts latch ERR_SPIN.
void launch_local_sort(hipStream_t st, uint64_t* keys, uint32_t* ids, const uint32_t* bstart, uint32_t nb,
                       const uint32_t* top, uint32_t* big, uint32_t* err, bool wide);
// Then the buckets of BUCKET_MAX + 1 .. BUCKET_HUGE pairs: each is sorted in
// LDS and its flag cleared, unless one of its sub-buckets holds more than the
// in-LDS scheme takes (then it is left untouched, flagged, for the segmented
// passes).
void launch_local_sort_huge(hipStream_t st, uint64_t* keys, uint32_t* ids, const uint32_t* bstart, uint32_t nb,
                            uint32_t* big);
// Tile counts of the big buckets: tile_off = exclusive scan of the tiles per
// bucket, big_idx = exclusive scan of big[]; totals[0] = tiles, totals[1] =
// big buckets. ntiles, tile_off, big_idx hold nb words; tmp 2 scan_tmp_words(nb).
void launch_big_tables(hipStream_t st, const uint32_t* bstart, const uint32_t* big, uint32_t nb, uint32_t* ntiles,
                       uint32_t* tile_off, uint32_t* big_idx, uint32_t* totals, uint32_t* tmp);
// Segment tables (segment = big bucket) for the segmented passes.
void launch_big_fill(hipStream_t st, const uint32_t* bstart, const uint32_t* big, const uint32_t* big_idx,
                     const uint32_t* tile_off, uint32_t nb, const SegTiles& sg, uint64_t* seg_begin);
// Per-segment histograms of the six low key digits: hist [num][8][256], zeroed.
// Over the first *ntiles tiles (at most max_tiles).
void launch_seg_hist_keys(hipStream_t st, const uint64_t* keys, uint64_t max_tiles, const uint32_t* ntiles,
                          const SegTiles& sg, uint32_t* hist);

// ------------------------------------------------------------------ scans
// Exclusive prefix sums; `total` (device, may be null) receives the sum.
// tmp needs scan_tmp_words(n) words.
uint64_t scan_tmp_words(uint64_t n);
// gate (device, may be null): if it reads 0 when the kernels run, they do
// nothing (outputs and total untouched).
void launch_scan_u32(hipStream_t st, const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total,
                     uint32_t* tmp, const uint32_t* gate = nullptr);
// Up to SCAN_MULTI independent scans (in[y] -> out[y], n[y] items, total[y]
// may be null) in one set of launches; tmp needs SCAN_MULTI times
// scan_tmp_words of the largest n[y]. An empty array gets total 0. With a
// gate as above.
constexpr int SCAN_MULTI = 4;
struct ScanSet {
    const uint32_t* in[SCAN_MULTI];
    uint32_t* out[SCAN_MULTI];
    uint32_t* total[SCAN_MULTI];
    uint64_t n[SCAN_MULTI];
    const uint32_t* gate = nullptr;
};
void launch_scan_multi(hipStream_t st, const ScanSet& s, int k, uint32_t* tmp);

// ------------------------------------------------------------------ build
// Fill leaves from sorted pairs: leaf j takes sorted positions
// [floor(j n / L), floor((j+1) n / L)), its points decoded from the keys;
// writes slot j, the pivot and the leaf record. Requires n / L <= 32.
// skip (device, may be null): the fill does nothing if it holds nonzero.
void launch_build_leaves(hipStream_t st, int dim, int curve, const uint64_t* sk, const uint32_t* sid,
                         uint64_t n, uint64_t L, uint32_t C, uint32_t* slots, uint64_t* piv_key,
                         uint32_t* piv_id, NodeRec* leafrec, const uint64_t* skip = nullptr);
// Every node level of the layout in dt, bottom up (parent i = union and sum
// of children [B i, B i + B)), several levels per launch. L_bound bounds the
// leaf count (the grids and the number of launches); levels above the
// tree's height do nothing.
void launch_node_levels(hipStream_t st, int dim, const DevTree* dt, const Dirs& dirs, uint64_t L_bound,
                        NodeRec* inner, uint32_t B);
// Every PSAMPLE-th pivot of the current directory, {key lo, key hi, id, 0}
// per record, at most cap records (ceil(L / PSAMPLE) are written).
constexpr uint32_t PSAMPLE = 32;
void launch_pivot_sample(hipStream_t st, const DevTree* dt, const Dirs& dirs, uint4* out, uint64_t cap);
// Packed boxes of the current leaves (leaves = true) or inner nodes of dt;
// cap bounds their number.
void launch_pack_tree(hipStream_t st, int dim, const DevTree* dt, const Dirs& dirs, bool leaves,
                      const NodeRec* inner, uint4* out, uint64_t cap);

// ---------------------------------------------------------------- queries


// What a query kernel needs of a tree. For a resident index `dt` is set and
// the kernels take leaf, pkey, L, h and the level table from it at launch
// (resolve_tree); the other fields are fixed per index. With dt == nullptr
// (many small indexes, exports after a sync) every field is taken as given.
struct TreeView {
    const NodeRec* inner;   // levels 0..h-1
    const NodeRec* leaf;    // level h (the directory); with dt: directory buffer 0
    const NodeRec* leaf_alt;  // with dt: directory buffer 1
    const uint4* cinner;    // packed boxes of inner (same positions)
    const uint4* cleaf;     // packed boxes of leaf
    const uint64_t* pkey;   // leaf pivot keys (ascending); with dt: buffer 0
    const uint64_t* pkey_alt;  // with dt: buffer 1
    const uint32_t* slots;
    uint32_t h;
    uint32_t B;
    uint32_t C;
    uint64_t L;
    const DevTree* dt;
};
#ifdef __HIPCC__
// The directory buffers come in as kernel arguments (leaf / leaf_alt, pkey /
// pkey_alt), so the compiler knows they are device memory and loads through
// them are global loads; the device state only says which one is current.
__device__ __forceinline__ TreeView resolve_tree(const TreeView& tv) {
    TreeView t = tv;
    if (tv.dt) {
        const DevTree* d = tv.dt;
        const bool c = d->cur != 0;
        t.leaf = c ? tv.leaf_alt : tv.leaf;
        t.pkey = c ? tv.pkey_alt : tv.pkey;
        t.L = d->L;
        t.h = d->h;
    }
    return t;
}
#endif
// Queries are processed in the order `order` gives (nullptr: input order);
// results always land in the query's own row.
// qkeys: curve keys of the queries in input order (seeds the search with the
// leaves around each query's own curve position). variant 0: seeded
// fixed-order traversal; 1: nearest-child-first traversal. hcap: an upper
// bound of the tree's height that sizes the seeded walk's stack of child
// masks in LDS (up to KNN_STACK_MAX levels; a taller tree walks without
// it). err: flags word (ERR_STACK if the tree outgrew hcap). stats
// (nullable): queries, box tests, leaves and points scanned are added to
// stats[0..3] (the seeded walks only).
constexpr uint32_t KNN_STACK_MAX = 24;
constexpr uint32_t KNN_CAND = 16;      // default: candidate leaves a seeded walk collects before scanning them
constexpr uint32_t KNN_CAND_MAX = 32;
// Runtime knobs of the lane-per-query seeded search (no effect on results):
// seed leaves (odd: the query's own leaf and (seed_leaves - 1) / 2 on each
// side in curve order) and the candidate list's length.
struct KnnTuning {
    uint32_t seed_leaves = 3;
    uint32_t cand = KNN_CAND;
};
void launch_knn(hipStream_t st, int dim, const TreeView& t, const uint32_t* q, const uint64_t* qkeys, uint64_t nq,
                const uint32_t* order, uint32_t k, int variant, uint32_t hcap, const KnnTuning& tune, uint32_t* err,
                unsigned long long* stats, uint32_t* ids, uint64_t* d2);
// Boxes are processed in the order `order` gives (nullptr: input order);
// results always land at the box's own index.
void launch_range_count(hipStream_t st, int dim, const TreeView& t, const uint32_t* boxes, uint64_t nb,
                        const uint32_t* order, uint64_t* counts);
void launch_range_report(hipStream_t st, int dim, const TreeView& t, const uint32_t* boxes, uint64_t nb,
                         const uint32_t* order, const uint64_t* offsets, uint32_t* ids);
// One thread per box (kept for comparison in tests and benchmarks).
void launch_range_count_lane(hipStream_t st, int dim, const TreeView& t, const uint32_t* boxes, uint64_t nb,
                             uint64_t* counts);

// ---------------------------------------------------------- P-Orth tree
// Nodes of the P-Orth tree (Sec. 3) in depth-first preorder, children in
// Morton order, as two arrays:
//   box[v]  (16 bytes): the exact bounding box of the node's points, packed
//           as for the kNN box tests (BoxBits: low corner in the first 64-bit
//           word, high corner in the second); bit 63 of the first word is set
//           for a leaf;
//   link[v] (8 bytes): interior {index one past its subtree, points below};
//           leaf {first of its points in the point array, count}.
constexpr uint32_t ORTH_TILE = 2048;  // sorted positions per block of the leaf marking

struct OrthView {
    const uint4* box;
    const uint2* link;
    const uint32_t* first;     // first point of each node's subtree
    const uint4* pts;          // {x, y, z or 0, id} in Morton order
    const uint32_t* ids;       // the same ids, alone
    const uint32_t* lstart;    // first point of each leaf, in leaf order
    const uint64_t* fkey;      // Morton key of each leaf's first point
    const uint8_t* llev;       // level of each leaf
    const uint32_t* base;      // preorder index of the first node each leaf opens
    uint64_t N;                // nodes
    uint32_t L;                // leaves
    uint32_t n;                // points
};
// Leaf cut of the sorted keys, first pass: per position a mark byte (leaf
// level, bit 7 = a leaf starts here; mark holds a whole number of tiles),
// the number of leaf starts of each ORTH_TILE tile, and every point {coords
// decoded from its key, id} (pts) and its id (ids).
void launch_orth_mark(hipStream_t st, int dim, const uint64_t* sk, const uint32_t* sid, uint64_t n, uint32_t phi,
                      uint8_t* mark, uint32_t* tile_cnt, uint4* pts, uint32_t* ids);
// Second pass, with tile_off the exclusive scan of the tile counts: each
// leaf's first position, level, first key and box (packed, leaf bit set).
void launch_orth_leaves(hipStream_t st, int dim, const uint64_t* sk, uint64_t n, const uint8_t* mark,
                        const uint32_t* tile_off, uint32_t* lstart, uint8_t* llev, uint64_t* fkey, uint4* lbox);
// Interior nodes that open at each leaf, plus one (cnt1, L words), and the
// largest leaf level (atomic max into *maxlev, zeroed first).
void launch_orth_counts(hipStream_t st, int dim, const uint8_t* llev, const uint64_t* fkey, uint32_t L,
                        uint32_t* cnt1, uint32_t* maxlev, uint32_t* err);
// Nodes in preorder from base = exclusive scan of cnt1 (N nodes in all):
// links and first points of every node, boxes of the leaves (lbox, in leaf
// order); lev[v] = level of interior node v, 0xFF for a leaf.
void launch_orth_nodes(hipStream_t st, int dim, const uint8_t* llev, const uint64_t* fkey, const uint32_t* lstart,
                       const uint32_t* base, uint32_t L, uint32_t n, uint64_t N, const uint4* lbox, uint4* box,
                       uint2* link, uint32_t* first, uint8_t* lev);
// Boxes of the interior nodes of one level from their children.
void launch_orth_boxes(hipStream_t st, int dim, uint32_t level, uint64_t N, const uint8_t* lev, uint4* box,
                       const uint2* link);
// Nodes as 8 words each: lo[3], hi[3], then link.x and link.y | 0x80000000
// for a leaf.
void launch_orth_export(hipStream_t st, int dim, const uint4* box, const uint2* link, uint64_t N, uint32_t* out);
// Queries over a P-Orth tree (k <= 128: a lane per query up to 16, else a
// wave; order and qkeys as for launch_knn).
void launch_orth_knn(hipStream_t st, int dim, const OrthView& t, const uint32_t* q, const uint64_t* qkeys,
                     uint64_t nq, const uint32_t* order, uint32_t k, uint32_t* ids, uint64_t* d2);
// counts (ids null) or reports into ids[offsets[b] .. offsets[b + 1]).
void launch_orth_range(hipStream_t st, int dim, const OrthView& t, const uint32_t* boxes, uint64_t nb,
                       const uint32_t* order, uint64_t* counts, const uint64_t* offsets, uint32_t* ids);

// P-Orth batch updates (the tree is canonical: the new set's sorted pairs are
// made from the old order, then the tree is cut again).
// place[j] = old points whose key is <= new key bk[j]; hist[place[j]] += 1
// (hist: n + 1 words, zeroed).
void launch_orth_place(hipStream_t st, int dim, const uint4* pts, uint64_t n, const uint64_t* bk, uint64_t m,
                       uint32_t* place, uint32_t* hist);
// Merged (key, id) pairs of the old points and the sorted batch into mk/mi
// (n + m); hscan = exclusive scan of hist over its first n words.
void launch_orth_merge(hipStream_t st, int dim, const uint4* pts, uint64_t n, const uint32_t* hist,
                       const uint32_t* hscan, const uint64_t* bk, const uint32_t* bid, const uint32_t* place,
                       uint64_t m, uint64_t* mk, uint32_t* mi);
// Clears the live bits of the batch's ids below next_id; *removed += bits
// that were set; keep[position of each removed point] = 0 (keep: n words,
// filled with 1 first; idkey: Morton key per id). A removed id not found in
// the point array latches ERR_ORTH.
void launch_orth_kill(hipStream_t st, int dim, const uint32_t* dids, uint64_t m, uint32_t next_id, uint32_t* alive,
                      const uint64_t* idkey, const uint4* pts, uint64_t n, uint32_t* keep,
                      unsigned long long* removed, uint32_t* err);
// Flagged points' (key, id) to mk/mi[pos[i]] (pos = exclusive scan of flag).
void launch_orth_compact(hipStream_t st, int dim, const uint4* pts, uint64_t n, const uint32_t* flag,
                         const uint32_t* pos, uint64_t* mk, uint32_t* mi);
// Sets the live bits of ids [lo, hi) (words past the one holding lo - 1 are
// written whole).
void launch_orth_alive(hipStream_t st, uint32_t* alive, uint32_t lo, uint32_t hi);
void launch_orth_put64(hipStream_t st, unsigned long long* p, unsigned long long v);

// ----------------------------------------------------------------- export
// Prefix sums of leaf counts -> entry offsets (u64, L+1 entries).
void launch_leaf_offsets(hipStream_t st, const NodeRec* leaf, uint64_t L, uint64_t* off, uint64_t* tmp);
void launch_export_sorted(hipStream_t st, int dim, int curve, const TreeView& t, const uint64_t* off,
                          uint64_t* keys, uint32_t* ids, uint32_t* pts);
void launch_export_raw(hipStream_t st, int dim, const TreeView& t, const uint64_t* off, uint32_t* ids,
                       uint32_t* pts);
void launch_export_structure(hipStream_t st, int dim, const TreeView& t, uint64_t n_inner,
                             const uint64_t* piv_key_src, const uint32_t* piv_id_src, uint64_t* piv_key,
                             uint32_t* piv_id, uint32_t* leaf_cnt, uint32_t* leaf_lo, uint32_t* leaf_hi,
                             uint32_t* node_lo, uint32_t* node_hi, uint64_t* node_cnt);

// ------------------------------------------------------------ many indexes
// Per-index tree metadata of a batch of independent indexes built together.
constexpr int MULTI_LEVELS = 26;
struct IdxMeta {
    uint32_t L, h, leaf_base, inner_base;  // leaves, height, first global leaf / inner node
    uint32_t n, pt_base, pad0, pad1;       // points and first global point
    uint32_t lvl_off[MULTI_LEVELS];        // first node of level l among the index's inner nodes
    uint32_t lvl_n[MULTI_LEVELS];          // nodes of level l (level h = the leaves)
};

// Encode + per-segment digit histograms, one block per tile (tile tables as in
// SegTiles); hist is [num][8][256], zeroed.
void launch_encode_hist_seg(hipStream_t st, int dim, int curve, const uint32_t* pts, uint64_t ntiles,
                            const SegTiles& sg, uint64_t* keys, uint32_t* hist, uint32_t* err);
// off[s][p][d] = seg_begin[s] + exclusive prefix over digits of hist[s][p][.]
void launch_seg_digit_offsets(hipStream_t st, uint32_t num, const uint32_t* hist, const uint64_t* seg_begin,
                              uint32_t* off, const uint32_t* num_dev = nullptr);
// Leaves of every index: global leaf g belongs to index s with
// leaf_off[s] <= g < leaf_off[s+1]; ids stored are local (position - pt_base).
void launch_build_leaves_seg(hipStream_t st, int dim, int curve, uint32_t num, uint64_t total_leaves,
                             const uint32_t* leaf_off, const IdxMeta* meta, const uint64_t* sk, const uint32_t* sid,
                             uint32_t C, uint32_t* slots, uint64_t* piv_key, uint32_t* piv_id, NodeRec* leafrec);
// Parents at height u (1 = parents of leaves) of every index with h >= u;
// pref[s] = number of such parents before index s (num + 1 entries).
void launch_node_step_seg(hipStream_t st, int dim, uint32_t num, uint64_t nparents, uint32_t u, const uint32_t* pref,
                          const IdxMeta* meta, const NodeRec* leafrec, NodeRec* inner, uint32_t B);
// kNN over many indexes in one persistent launch; work items are (index,
// chunk of 64 queries) taken from an atomic counter (zeroed before launch).
// hcap: the tallest index's height (sizes the walk's stack in LDS).
void launch_multi_knn(hipStream_t st, int dim, int curve, const TreeView& tv, const IdxMeta* meta, uint32_t num,
                      const uint64_t* q_off, const uint32_t* q, uint32_t* chunk_pref, uint32_t* work_ctr, uint32_t k,
                      uint32_t hcap, uint32_t* ids, uint64_t* d2, uint32_t* tmp, uint32_t* err);

}  // namespace psi
