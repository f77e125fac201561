/* psi.h -- C ABI of the MI355X (gfx950) SPaC-tree library.
 *
 * A SPaC-tree ("Parallel Dynamic Spatial Indexes", PPoPP'26, Sec. 4) is a
 * spatial index over 2D/3D integer points ordered by a space-filling-curve
 * key (Morton = SPaC-Z, Hilbert = SPaC-H). Points live in leaf blocks of at
 * most `leaf_size` entries at build time; leaves keep no internal order
 * (Sec. 4.2, "relaxing the key order in the leaves"); every leaf and every
 * tree node stores the tight axis-aligned box of its points (Sec. 1, App. C).
 *
 * Conventions shared by every call
 *   - Every pointer named d_* is DEVICE memory owned by the caller; it must
 *     stay valid until the work queued on the index's stream has finished.
 *     Host pointers are named h_* .
 *   - Calls are asynchronous and ordered on the stream given to psi_create
 *     (or psi_set_stream). Argument errors are returned at once. Errors that
 *     only the device can see (coordinate out of range, an internal check)
 *     are latched and returned by the next psi_sync / psi_size.
 *   - Build, insert, delete and the queries only enqueue work: none of them
 *     waits for the stream. The sizes of the tree (leaf count, current
 *     directory, slots, next id, node layout) live in device memory and are
 *     planned, checked and committed by kernels; the host sizes buffers and
 *     grids by upper bounds (an update's worst case for its batch size), which
 *     it tightens from a copy of the device state taken after each update
 *     without waiting for it. A call may still wait when more than 64 updates
 *     are queued, when two or more queued updates could together have grown
 *     the tree past 1.5 times its last known size (their worst cases add up;
 *     the oldest is waited for), or when a replayed graph left the sizes
 *     unknown. Growing a
 *     buffer never waits either (the replaced block is freed once the stream
 *     is idle). The inspection calls (psi_sync, psi_size, psi_next_id,
 *     psi_shape, the exports) wait for the stream.
 *   - Points are row-major uint32 [n][dim]. 2D coordinates must be < 2^31 and
 *     3D coordinates < 2^21: the key has 32 (2D) or 21 (3D) bits per axis
 *     (Sec. 3, the precision a 64-bit code allows), and 2D squared distances
 *     must fit 64 bits.
 *   - Boxes are uint32 [nb][2][dim]: the lo row, then the hi row; both ends
 *     are inclusive. A box with lo > hi in any axis is empty.
 *   - Ids are uint32 assigned by the library: psi_build numbers its points
 *     0..n-1 in input order; each insert continues from the next unused id.
 *     Ids are never reused.
 *   - An index is bound to one stream and is not thread-safe.
 */
#ifndef PSI_H
#define PSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSI_OK = 0,
    PSI_E_ARG = 1,       /* bad argument (null pointer, bad size or parameter) */
    PSI_E_RANGE = 2,     /* a coordinate exceeds the key's bits per axis */
    PSI_E_NOMEM = 3,     /* device allocation failed */
    PSI_E_CAPACITY = 4,  /* id space (2^32 - 1 ids) exhausted, or an update did not fit
                            the buffers a captured graph was sized with */
    PSI_E_HIP = 5,       /* a HIP runtime call failed */
    PSI_E_STATE = 6,     /* call not valid in the index's current state */
    PSI_E_INTERNAL = 7   /* a device-side consistency check failed */
} psi_status;

typedef enum { PSI_MORTON = 0, PSI_HILBERT = 1 } psi_curve;

/* psi_params.flags bits. By default a query batch of 4096 or more queries
 * (or boxes) is processed in curve-key order of its points (box centres) so
 * that neighbouring queries share tree nodes; results are the same either
 * way. PSI_FLAG_INPUT_ORDER processes batches in input order.
 * kNN with k <= 16 runs one query per lane. By default each search is
 * seeded with the leaves around the query's own curve key and then walks the
 * tree in fixed child order, pruning by the k-th distance;
 * PSI_FLAG_KNN_NEAREST_FIRST instead descends to the nearest child first and
 * re-scores siblings on the way back (App. C's visiting order). Both return
 * the same exact result.
 * A build of 2^24 or more points sorts its (key, id) pairs in two levels:
 * two global radix passes on the top 16 key bits, then each bucket in one
 * workgroup's local memory (the distribute-then-sort-locally shape of
 * Alg. 3); smaller builds take eight global passes. PSI_FLAG_SORT_BUCKETS and
 * PSI_FLAG_SORT_LSD force one or the other (not both); the result is the
 * same.
 * Leaves keep their entries unsorted after inserts (Sec. 4.2: an insert
 * appends to its leaf; only a leaf that is re-cut is sorted).
 * PSI_FLAG_SORTED_LEAVES keeps every leaf in (key, id) order after every
 * update instead, the total order a CPAM-style tree maintains (Sec. 4 and
 * Sec. 5.1.2 compare the two): each insert re-sorts the leaves it appended
 * to. Query results and the set are the same; only update cost differs. */
enum {
    PSI_FLAG_INPUT_ORDER = 1,
    PSI_FLAG_KNN_NEAREST_FIRST = 2,
    PSI_FLAG_SORT_BUCKETS = 4,
    PSI_FLAG_SORT_LSD = 8,
    PSI_FLAG_SORTED_LEAVES = 16
};

/* dim: 2 or 3. curve: psi_curve. leaf_size: phi, the largest leaf a build
 * makes (2..32); a leaf slot holds 2*phi entries so that inserts can append
 * without moving data. fanout: children per tree node (2..32). flags: a
 * combination of PSI_FLAG_* bits. */
typedef struct {
    uint32_t dim;
    uint32_t curve;
    uint32_t leaf_size;
    uint32_t fanout;
    uint32_t flags;
} psi_params;

typedef struct psi_index_s* psi_index;
typedef struct psi_multi_s* psi_multi;
typedef struct psi_graph_s* psi_graph;

const char* psi_status_str(psi_status s);

/* Create an empty index bound to `hip_stream` (a hipStream_t; NULL = the
 * default stream). */
psi_status psi_create(const psi_params* prm, void* hip_stream, psi_index* out);
psi_status psi_destroy(psi_index ix);
psi_status psi_set_stream(psi_index ix, void* hip_stream);

/* Build (Alg. 3): replace the contents with the n points d_pts, ids 0..n-1.
 * Encodes each point's curve key, sorts the (key, id) pairs, cuts the sorted
 * order into ceil(n/phi) balanced leaves and builds the node levels above.
 * The resulting structure is canonical (a function of the point set only). */
psi_status psi_build(psi_index ix, const uint32_t* d_pts, uint64_t n);

/* Batch insert (Alg. 4): add m points; their ids are the next m unused ids
 * in input order, written to d_new_ids (may be NULL). Each sorted run of new
 * points is appended, unsorted, to the leaf whose key range holds it; a leaf
 * that would exceed 2*phi entries is re-cut into balanced leaves. A batch with
 * a coordinate out of range is rejected whole on the device before any leaf
 * changes: nothing is inserted, no id is used, d_new_ids reads 0xFFFFFFFF and
 * the next psi_sync returns PSI_E_RANGE. */
psi_status psi_batch_insert(psi_index ix, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids);

/* Batch delete (Sec. 4.2): remove the live points whose ids are listed.
 * Unknown, already deleted and repeated ids are ignored. The number removed
 * is written to *d_ndeleted (device uint64; may be NULL). Leaves that fall
 * below ceil(phi/2) entries are merged with their right neighbour (the left
 * one at the end) and re-cut. */
psi_status psi_batch_delete(psi_index ix, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted);

/* k nearest neighbours (Sec. 2.2) of nq query points, exact: row q of
 * d_ids/d_d2 ([nq][k]) holds the k live points with the smallest (squared
 * Euclidean distance, id), ascending; rows are padded with
 * (0xFFFFFFFF, UINT64_MAX) when the index has fewer than k points.
 * 1 <= k <= 128. Query coordinates obey the same limits as points (a query
 * out of range latches PSI_E_RANGE). */
psi_status psi_knn(psi_index ix, const uint32_t* d_q, uint64_t nq, uint32_t k,
                   uint32_t* d_ids, uint64_t* d_d2);

/* Range count (Sec. 2.2): d_counts[b] = number of live points in box b. */
psi_status psi_range_count(psi_index ix, const uint32_t* d_boxes, uint64_t nb, uint64_t* d_counts);

/* Range list (Sec. 2.2): ids of the live points in box b are written to
 * d_ids[d_offsets[b] .. d_offsets[b+1]), in an unspecified but deterministic
 * order. d_offsets ([nb+1], device) is normally the exclusive prefix sum of
 * psi_range_count's output; a box whose span is shorter than its count is
 * truncated to its span. */
psi_status psi_range_report(psi_index ix, const uint32_t* d_boxes, uint64_t nb,
                            const uint64_t* d_offsets, uint32_t* d_ids);

/* Waits for the stream; returns the first latched device error, if any
 * (PSI_E_RANGE; PSI_E_CAPACITY for an update a replayed graph could not fit
 * into the buffers it was captured with; PSI_E_INTERNAL), and clears it. */
psi_status psi_sync(psi_index ix);
/* Number of live points (waits for the stream, like psi_sync). */
psi_status psi_size(psi_index ix, uint64_t* h_n_live);
/* Next id that an insert would assign (waits for the stream). */
psi_status psi_next_id(psi_index ix, uint32_t* h_next_id);

/* --- inspection (tests, checkpoints) ------------------------------------ */

/* All live entries in (key, id) order: d_keys [n], d_ids [n], d_pts [n][dim]
 * (any may be NULL). Leaves are sorted on the fly; the index is unchanged. */
psi_status psi_export(psi_index ix, uint64_t* d_keys, uint32_t* d_ids, uint32_t* d_pts);

/* Tree shape: number of leaves, height h (levels 0..h, level h = leaves) and
 * the node count of each level in h_level_sizes[0..h] (at most 64 levels). */
psi_status psi_shape(psi_index ix, uint64_t* h_n_leaves, uint32_t* h_height, uint64_t* h_level_sizes);

/* Leaves and nodes. Leaf j: pivot (key, id) -- a lower bound of its entries
 * that is strictly above every entry of leaf j-1 --, entry count, and tight
 * box [L][dim]. Nodes of all levels, root first and leaves last, with their
 * boxes [nodes][dim] and counts. Any pointer may be NULL. */
psi_status psi_export_structure(psi_index ix, uint64_t* d_piv_key, uint32_t* d_piv_id,
                                uint32_t* d_leaf_cnt, uint32_t* d_leaf_lo, uint32_t* d_leaf_hi,
                                uint32_t* d_node_lo, uint32_t* d_node_hi, uint64_t* d_node_cnt);

/* Raw leaf contents in leaf order, entries in their stored (unsorted) order:
 * d_ids [n], d_pts [n][dim]. Leaf j's entries start at the exclusive prefix
 * sum of the leaf counts. */
psi_status psi_export_leaves(psi_index ix, uint32_t* d_ids, uint32_t* d_pts);

/* --- single steps of the path (parity tests, micro-benchmarks) ------------ */

/* Curve keys of n points (Sec. 2.2): d_keys[i] = key of d_pts[i]. */
psi_status psi_encode(uint32_t dim, uint32_t curve, const uint32_t* d_pts, uint64_t n,
                      uint64_t* d_keys, void* hip_stream);

/* Stable sort of n (key, id) pairs by (key, id) (Alg. 3 sorts pairs, not
 * points). Inputs are left unchanged; outputs go to d_keys_out/d_ids_out.
 * Temporary device memory is allocated and freed inside the call, which
 * therefore waits on the stream before returning. */
psi_status psi_sort_pairs(const uint64_t* d_keys, const uint32_t* d_ids, uint64_t n,
                          uint64_t* d_keys_out, uint32_t* d_ids_out, void* hip_stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * sort as psi_sort_pairs, with the same result, but no allocation and no
 * wait. Its workspace is a fixed device array of about 25 MB inside the
 * library, one per GPU, kept until the process ends; n above
 * PSI_SORT_NOALLOC_MAX returns PSI_E_ARG and queues nothing. Every call on
 * one GPU shares that GPU's workspace, so calls that may run at the same time
 * on one GPU (on different streams) race; calls on one stream are safe. The
 * outputs must not overlap the inputs. */
#define PSI_SORT_NOALLOC_MAX (1u << 20)
psi_status psi_sort_pairs_noalloc(const uint64_t* d_keys, const uint32_t* d_ids, uint64_t n,
                                  uint64_t* d_keys_out, uint32_t* d_ids_out, void* hip_stream);

/* --- many independent indexes (batched small indexes) -------------------- */

/* Build `num` independent indexes from one CSR batch: index s holds the
 * points d_pts[d_pt_off[s] .. d_pt_off[s+1]) (d_pt_off: device uint64
 * [num+1], d_pt_off[0] = 0) with local ids 0.. in that order. All indexes are
 * encoded, sorted (one segment per index), cut into leaves and given their
 * node levels by the same launches; each index's structure equals what
 * psi_build makes from its points alone. At most 2^24 points per index and
 * 2^32 - 1 in total. Waits on the stream (the offsets are read on the host). */
psi_status psi_multi_build(const psi_params* prm, void* hip_stream, uint32_t num, const uint64_t* d_pt_off,
                           const uint32_t* d_pts, psi_multi* out);
psi_status psi_multi_destroy(psi_multi mx);
/* kNN (as psi_knn) of query batches of uneven sizes: the queries
 * d_q[d_q_off[s] .. d_q_off[s+1]) search index s; rows of d_ids/d_d2
 * ([total queries][k]) follow d_q. All batches run in ONE persistent launch
 * whose waves take (index, 64-query chunk) items from an atomic counter.
 * k in {1, 2, 4, 8, 10, 16}. Never waits on the stream. */
psi_status psi_multi_knn(psi_multi mx, const uint64_t* d_q_off, const uint32_t* d_q, uint32_t k,
                         uint32_t* d_ids, uint64_t* d_d2);
/* Waits for the stream; returns the first latched device error. */
psi_status psi_multi_sync(psi_multi mx);
/* Shape and structure of index `index` (as psi_shape / psi_export_structure). */
psi_status psi_multi_shape(psi_multi mx, uint32_t index, uint64_t* h_n_leaves, uint32_t* h_height,
                           uint64_t* h_level_sizes);
psi_status psi_multi_export_structure(psi_multi mx, uint32_t index, uint64_t* d_piv_key, uint32_t* d_piv_id,
                                      uint32_t* d_leaf_cnt, uint32_t* d_leaf_lo, uint32_t* d_leaf_hi,
                                      uint32_t* d_node_lo, uint32_t* d_node_hi, uint64_t* d_node_cnt);
/* Entries of every index, index by index, each in (key, id) order (local
 * ids); lengths follow the build's offsets. */
psi_status psi_multi_export(psi_multi mx, uint64_t* d_keys, uint32_t* d_ids, uint32_t* d_pts);

/* --- serving: continuous batching of mixed requests ----------------------- */

/* A server takes over a resident index and serves a stream of requests by
 * continuous batching (the paper's operations under a request load; the
 * consistency rule is sequential consistency in submission order: every
 * request sees exactly the updates submitted before it, as if the requests
 * ran one at a time).
 *   - Requests are grouped into epochs, maximal runs of updates or of
 *     queries, admitted in submission order while the sum of their estimated
 *     device footprints stays within budget_bytes (a request that could never
 *     fit is refused with PSI_E_CAPACITY; when the budget is full, the
 *     oldest epoch is waited for).
 *   - Consecutive inserts run as one batch (ids in submission order, as
 *     separate inserts would give them). kNN requests of one epoch with the
 *     same k run as one launch.
 *   - Updates run on one stream of the server's, queries on another. An
 *     update's encode, sort, routing and planning overlap the queries of the
 *     epoch before it; its first change to the tree waits for them. A query
 *     epoch waits for the updates before it.
 *   - psi_server_submit queues a request and returns a ticket at once;
 *     psi_server_poll and psi_server_flush dispatch queued epochs (without
 *     waiting for the device, unless the budget is full); psi_server_wait
 *     dispatches and waits for one ticket.
 *   - The index must not be used directly while the server exists; it gets
 *     its stream back when the server is destroyed.
 * Every d_* buffer is device memory owned by the caller and must stay valid,
 * and the inputs unchanged, until the request's ticket is done. */
enum {
    PSI_REQ_INSERT = 0,        /* d_in: points [n][dim]; d_ids: new ids [n] (may be NULL) */
    PSI_REQ_DELETE = 1,        /* d_in: ids [n]; d_out: number removed [1] (may be NULL) */
    PSI_REQ_KNN = 2,           /* d_in: queries [n][dim]; k; d_ids [n][k], d_out: d2 [n][k] (as psi_knn) */
    PSI_REQ_RANGE_COUNT = 3,   /* d_in: boxes [n][2][dim]; d_out: counts [n] */
    PSI_REQ_RANGE_REPORT = 4   /* d_in: boxes; d_out: offsets [n+1] (exclusive scan of the counts);
                                  d_ids: ids [ids_cap]; a box's ids past ids_cap are dropped (the
                                  offsets still give the true counts) */
};
typedef struct {
    uint32_t kind;          /* PSI_REQ_* */
    uint32_t k;             /* kNN only: 1..128 */
    uint64_t n;             /* points, ids, queries or boxes */
    const uint32_t* d_in;
    uint32_t* d_ids;
    uint64_t* d_out;
    uint64_t ids_cap;       /* range report only */
    void* ready_event;      /* hipEvent_t the server waits for before reading d_in (may be NULL) */
} psi_request;
typedef struct psi_server_s* psi_server;

psi_status psi_server_create(psi_index ix, uint64_t budget_bytes, psi_server* out);
/* Dispatches what is queued, waits for everything, gives the index back. */
psi_status psi_server_destroy(psi_server s);
psi_status psi_server_submit(psi_server s, const psi_request* req, uint64_t* h_ticket);
/* *h_done = 1 once the ticket's work has completed on the device; then
 * *h_done_ms (may be NULL) is its completion time in ms after
 * psi_server_create. Returns the ticket's status once done. */
psi_status psi_server_poll(psi_server s, uint64_t ticket, int* h_done, double* h_done_ms);
psi_status psi_server_wait(psi_server s, uint64_t ticket, double* h_done_ms);
psi_status psi_server_flush(psi_server s);

/* --- graph capture of index steps ----------------------------------------- */

/* Capture the calls (psi_build, psi_batch_insert, psi_batch_delete,
 * psi_knn, psi_range_count, psi_range_report, psi_multi_knn) issued on
 * `hip_stream` between psi_graph_begin and psi_graph_end into a hipGraph;
 * psi_graph_launch replays them with the same buffers and sizes.
 *   - Inside a capture no memory is allocated: run the same calls once with
 *     the same sizes before capturing (a call that would need a larger buffer
 *     returns PSI_E_STATE).
 *   - Every replay starts from the index's state at that moment: a captured
 *     insert hands out fresh ids on each replay (the next id is device
 *     state), a captured build resets the index. The per-leaf launches of a
 *     captured update cover as many leaves as the buffers hold; a replay
 *     that would exceed the buffers (or find more leaves than that) is
 *     refused on the device before it changes anything (the next psi_sync
 *     returns PSI_E_CAPACITY).
 *   - A graph records the indexes it touches. Any later eager build, update,
 *     or buffer growth of such an index stales the graph: psi_graph_launch
 *     then returns PSI_E_STATE and launches nothing (the graph would read a
 *     stale directory or freed memory). Replays themselves do not stale it.
 *   - After a replay that ran updates, the next call that needs the sizes
 *     (an update, an inspection call) waits for the stream once. */
psi_status psi_graph_begin(void* hip_stream);
psi_status psi_graph_end(void* hip_stream, psi_graph* out);
psi_status psi_graph_launch(psi_graph g, void* hip_stream);
psi_status psi_graph_destroy(psi_graph g);

/* --- P-Orth tree (Sec. 3) ---------------------------------------------- */

/* A second index kind: the parallel orth-tree of Sec. 3 (a quadtree in 2D,
 * an octree in 3D). Every node is a cell of the regular grid hierarchy over
 * the coordinate domain [0, 2^W)^D (W = 31 in 2D, 21 in 3D; the same
 * coordinate limits as psi_build): a cell is split at its midpoint on every
 * axis (the spatial median), so it has up to 2^D children, one per non-empty
 * sub-cell. A cell with more than leaf_size points is an interior node; a
 * cell with at most leaf_size points is a leaf, and so is a one-point cell
 * holding more (equal points cannot be split). This is the tree Alg. 1
 * builds after merging every subtree of at most leaf_size points into a
 * leaf; its shape does not depend on the skeleton height of Alg. 1. Boxes are
 * the exact bounding boxes of the points below each node.
 * Batch updates give the tree of the new point set (the tree is canonical, so
 * this is what Alg. 2's insertion and its deletion with flattening produce);
 * they reach it by merging the sorted batch into the sorted order of the old
 * points (or compacting that order) and cutting the tree again, in time
 * linear in the tree's size, not by Alg. 2's local sieve. */
typedef struct psi_orth_s* psi_orth;

/* prm: dim 2 or 3, curve must be PSI_MORTON (the tree's child order),
 * leaf_size 2..32, fanout ignored, flags a subset of PSI_FLAG_INPUT_ORDER,
 * PSI_FLAG_SORT_BUCKETS, PSI_FLAG_SORT_LSD (as for psi_create). Queries and
 * builds run on hip_stream. */
psi_status psi_orth_create(const psi_params* prm, void* hip_stream, psi_orth* out);
psi_status psi_orth_destroy(psi_orth o);

/* Builds the tree over n points (device, n x dim u32, row major; ids are
 * positions 0..n-1), replacing the previous tree. n < 2^31. Waits for the
 * stream twice (leaf and node counts). PSI_E_RANGE (and an empty tree) if a
 * coordinate is out of range. Not under graph capture (PSI_E_STATE).
 * Builds, inserts and deletes first return (and clear) an error latched by
 * an earlier call, as psi_orth_sync would, leaving the tree unchanged. */
psi_status psi_orth_build(psi_orth o, const uint32_t* d_pts, uint64_t n);

/* Inserts m points (device, m x dim u32); they get ids next_id ..
 * next_id + m - 1 in input order, written to d_new_ids (device, m u32) if
 * not null. PSI_E_RANGE (nothing inserted, tree unchanged) if a coordinate is
 * out of range; PSI_E_CAPACITY past 2^32 - 1 ids or 2^31 points. Waits for the
 * stream. Any other failure leaves the tree empty, with ids restarting at 0
 * (as does a failed delete). */
psi_status psi_orth_batch_insert(psi_orth o, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids);
/* Deletes the points with the given ids (device, m u32, any order); unknown,
 * deleted and repeated ids are ignored. *d_ndeleted (device u64, may be null)
 * receives the number removed. Waits for the stream. */
psi_status psi_orth_batch_delete(psi_orth o, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted);
/* Live points and the next id an insert hands out. */
psi_status psi_orth_size(psi_orth o, uint64_t* h_n_live, uint32_t* h_next_id);

/* Exact k nearest neighbours (k = 1..128), output as psi_knn. */
psi_status psi_orth_knn(psi_orth o, const uint32_t* d_q, uint64_t nq, uint32_t k, uint32_t* d_ids,
                        uint64_t* d_d2);
/* Points inside closed boxes (nb x [lo[dim], hi[dim]]), as psi_range_count
 * and psi_range_report; a report lists each box's ids in no particular
 * order. */
psi_status psi_orth_range_count(psi_orth o, const uint32_t* d_boxes, uint64_t nb, uint64_t* d_counts);
psi_status psi_orth_range_report(psi_orth o, const uint32_t* d_boxes, uint64_t nb, const uint64_t* d_offsets,
                                 uint32_t* d_ids);

/* Waits for the stream; returns and clears a latched error as psi_sync. */
psi_status psi_orth_sync(psi_orth o);

/* Node count, leaf count and height (levels of the deepest leaf + 1; 0 for
 * an empty tree). */
psi_status psi_orth_shape(psi_orth o, uint64_t* h_nodes, uint64_t* h_leaves, uint32_t* h_height);

/* Copies the tree out (either pointer may be null). d_nodes: nodes x 8 u32 in
 * depth-first preorder, children in Morton order: lo[3], hi[3] (the third
 * axis 0 in 2D), then for an interior node (index one past its subtree,
 * points below it) and for a leaf (first point, count | 0x80000000).
 * d_pts: n x 4 u32 {x, y, z or 0, id}, leaves' points contiguous, in the
 * order leaves appear. */
psi_status psi_orth_export(psi_orth o, uint32_t* d_nodes, uint32_t* d_pts);

/* Timing of the tree's kernels, as psi_prof_* (families "orth_marks",
 * "orth_nodes", "orth_boxes", "orth_merge", "orth_knn", "orth_range_count",
 * "orth_range_report", plus the sort's). */
psi_status psi_orth_prof_enable(psi_orth o, int on);
psi_status psi_orth_prof_reset(psi_orth o);
psi_status psi_orth_prof_get(psi_orth o, const char* family, double* h_ms, uint64_t* h_launches,
                             uint64_t* h_bytes);

/* --- kernel timing ------------------------------------------------------ */

/* When enabled, every kernel launch of the index is bracketed by HIP events
 * on its stream. psi_prof_get waits for the stream and returns, for the
 * named kernel family ("radix_pass", "encode_hist", "leaf_fill",
 * "leaf_meta", "nodes", "knn", "range_count", "range_report", "route",
 * "update", ...), the summed device time in ms, the launch count, and
 * the algorithmic bytes those launches move. psi_prof_reset clears them. */
psi_status psi_prof_enable(psi_index ix, int on);
/* Restricts the bracketing to one family (family: a NUL-terminated name,
 * copied), or lifts the restriction (family NULL): fewer events on the
 * stream while one kernel is timed. Other families then accumulate nothing.
 * PSI_E_ARG if ix is NULL. */
psi_status psi_prof_only(psi_index ix, const char* family);
psi_status psi_prof_reset(psi_index ix);
psi_status psi_prof_get(psi_index ix, const char* family, double* h_ms, uint64_t* h_launches,
                        uint64_t* h_bytes);

/* --- the SPaC-tree in the paper's own shape (Sec. 4) ---------------------
 * A binary search tree on (curve key, id): a subtree of at most leaf_wrap
 * points is one leaf (its entries in no particular order once appended to),
 * every interior node holds one point, its pivot, and has two children.
 * Boxes are tight (an interior node's covers its pivot). The paper sets
 * leaf_wrap = 40 (App. C); 2 <= leaf_wrap <= 64 here.
 *   - psi_bst_build: Alg. 3's BuildSorted over the points sorted by (key, id):
 *     a leaf when n <= leaf_wrap, else entry m = n / 2 is the pivot, [0, m)
 *     the left subtree and [m + 1, n) the right one.
 *   - psi_bst_batch_insert / psi_bst_batch_delete: Alg. 4's join-based
 *     recursion over the batch sorted by (key, id): a leaf takes its share
 *     unsorted while it fits leaf_wrap, is rebuilt by BuildSorted with it
 *     below 4 leaf_wrap points (App. C), else is exposed and the share goes
 *     on down; every node on the way joins its updated sides with Join
 *     (weight balance with alpha = 0.2: the lighter side weighs at least a
 *     fifth of both, weight = size + 1; single and double rotations; Node()
 *     turns a subtree of at most 2 leaf_wrap points into one or two leaves),
 *     or with Join2 when its pivot is deleted.
 *   - Queries, ids and errors behave as for psi_index (ids 0..n-1 at build,
 *     new ids from next_id on insert; unknown, dead and repeated ids are
 *     ignored on delete; kNN k <= 16).
 *   - Builds and updates wait for their work (they read counts back). An
 *     update is functional: a pool that runs out mid-way is grown and the
 *     update run again from the same root. Insert before any build:
 *     PSI_E_STATE. */
typedef struct psi_bst_s* psi_bst;
psi_status psi_bst_create(uint32_t dim, uint32_t curve, uint32_t leaf_wrap, void* hip_stream, psi_bst* out);
psi_status psi_bst_destroy(psi_bst t);
psi_status psi_bst_build(psi_bst t, const uint32_t* d_pts, uint64_t n);
psi_status psi_bst_batch_insert(psi_bst t, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids);
psi_status psi_bst_batch_delete(psi_bst t, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted);
psi_status psi_bst_knn(psi_bst t, const uint32_t* d_q, uint64_t nq, uint32_t k, uint32_t* d_ids, uint64_t* d_d2);
psi_status psi_bst_range_count(psi_bst t, const uint32_t* d_boxes, uint64_t nb, uint64_t* d_counts);
psi_status psi_bst_range_report(psi_bst t, const uint32_t* d_boxes, uint64_t nb, const uint64_t* d_offsets,
                                uint32_t* d_ids);
psi_status psi_bst_sync(psi_bst t);
/* Points n, the root reference (a node index, or a leaf index with bit 31
 * set) and the pool slots in use (node_slots interior-node records,
 * leaf_slots leaf records; freed slots among them are unreachable). */
psi_status psi_bst_shape(psi_bst t, uint64_t* h_n, uint32_t* h_root, uint64_t* h_node_slots, uint64_t* h_leaf_slots);
/* Device copies of the pools: d_nodes node_slots records of 16 words (lo[3],
 * size, hi[3], pivot id, pivot key (2 words, low first), left, right,
 * pivot point[3], 0), d_leaves leaf_slots records of 8 words (lo[3], count,
 * hi[3], sorted), d_ids leaf_slots x leaf_wrap ids and d_pts leaf_slots x
 * leaf_wrap points (D words each); a leaf's entries are the first count of
 * its slot. Unused coordinate words (2D) are 0. */
psi_status psi_bst_export(psi_bst t, uint32_t* d_nodes, uint32_t* d_leaves, uint32_t* d_ids, uint32_t* d_pts);

/* --- runtime knobs (for a tuner) ---------------------------------------- */

/* Knobs that change speed, never results. knn_seed_leaves: leaves scanned
 * before the walk of the lane-per-query kNN (k <= 16, the default
 * traversal): the query's own leaf (the last whose pivot key is not above
 * the query's curve key, App. C's nearby start) and (knn_seed_leaves - 1) / 2
 * on each side in curve order; odd, 1..9, default 3. knn_cand: candidate
 * leaves that walk collects before scanning them, 1..32, default 16.
 * order_bits: top curve-key bits the ordering of query and box batches sorts
 * on (8, 16, 24 or 32; default 24), when batches are ordered at all (not
 * with PSI_FLAG_INPUT_ORDER). psi_set_tuning returns PSI_E_ARG for values
 * out of range and changes nothing then; it applies to later calls. */
typedef struct psi_tuning {
    uint32_t knn_seed_leaves;
    uint32_t knn_cand;
    uint32_t order_bits;
} psi_tuning;
psi_status psi_set_tuning(psi_index ix, const psi_tuning* t);
psi_status psi_get_tuning(psi_index ix, psi_tuning* t);

/* Work counts of the kNN searches (App. C's visiting rule made measurable).
 * While enabled, every psi_knn of the index with the seeded traversal (the
 * default; not PSI_FLAG_KNN_NEAREST_FIRST) adds to four device counters:
 * queries answered, box tests (a node's bounding box read and compared with
 * the current k-th distance), leaves scanned and points scanned, seed leaves
 * included. enable: 1 starts counting from zero (when off before; allocates
 * 32 bytes, so not under graph capture: PSI_E_STATE), 0 stops. h_counts
 * (nullable, host, 4 entries): the counts so far, read after waiting for the
 * stream; all zero when counting was off. Counting adds a few atomic adds
 * per wave; timed runs leave it off. */
psi_status psi_query_stats(psi_index ix, int enable, uint64_t* h_counts);

#ifdef __cplusplus
}
#endif
#endif /* PSI_H */
