// Batch insert and delete kernels (Alg. 4 and Sec. 4.2).
//
// Updates work leaf by leaf on the sorted batch. Each batch entry is routed to
// the leaf whose pivot range holds its (key, id); entries of one leaf form a
// contiguous run of the sorted batch.
//  * insert: a run that fits the leaf's slot (2 phi entries) is appended
//    without sorting (the SPaC-tree's relaxed leaf order, Alg. 4). A leaf
//    that would overflow is merged with its run in (key, id) order and re-cut
//    into ceil(t / phi) balanced leaves, in fresh slots (the paper's local
//    rebuild of an overflowing leaf; App. C).
//  * delete: matching entries are removed from their leaf in place; the
//    leaf's box is recomputed exactly. Leaves that fall below ceil(phi/2)
//    entries are regrouped with the following leaves up to the next leaf that
//    is still full enough (the last group also takes the trailing under-full
//    leaves) and re-cut the same way; this keeps the leaf-size invariant that
//    Alg. 4's Node() restores by flattening or redistributing.
// Counters shared between kernels live in a small device array:
//   ctr[0] valid batch entries, [1] runs, [2] new leaf count, [3] slots to
//   allocate, [4] output chunks, [5] slots freed, [6] groups, [7] 1 + index
//   of the last full-enough leaf, [8] nonzero if a delete left a leaf below
//   the minimum (only then do leaves regroup), [9] range error of the
//   inserted batch, [10] outcome of the plan check (0 apply, 1 rejected,
//   2 the index was empty: the batch is built as a fresh tree), and the
//   64-bit word at [12] is nonzero unless that fresh build runs.
// Every size an update depends on (leaf count, slots, the free stack, the
// current directory buffer) is read from the index's device state (DevTree)
// and from these counters: the host sizes grids and buffers by upper bounds
// only, and the last kernel of the update commits the new state.
#include "psi_hilbert.h"
#include "psi_kern.h"
#include "psi_update.h"

namespace psi {

namespace {

inline unsigned blocks_for(uint64_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

// largest r in [0, R) with off[r] <= x (off ascending, off[0] == 0)
__device__ __forceinline__ uint32_t find_owner(const uint32_t* off, uint32_t R, uint64_t x) {
    uint32_t lo = 0, hi = R;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_route(const uint64_t* __restrict__ bk, const uint32_t* __restrict__ bi, uint64_t n,
                        const uint32_t* __restrict__ n_dev, const DevTree* __restrict__ dt,
                        uint32_t* __restrict__ leaf_of, Dirs dirs) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t ne = n_dev ? *n_dev : n;
    if (e >= ne) return;
    const uint32_t c = dt->cur;
    const uint64_t* pk = dirs.pkey[c];
    const uint32_t* pi = dirs.pid[c];
    const uint64_t L = dt->L;
    const uint64_t k = bk[e];
    const uint32_t i = bi[e];
    uint64_t lo = 0, hi = L;  // first pivot greater than (k, i); ids read on key ties only
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        const uint64_t km = pk[mid];
        const bool below = k < km || (k == km && i < pi[mid]);
        if (!below) lo = mid + 1;
        else hi = mid;
    }
    leaf_of[e] = lo == 0 ? 0u : (uint32_t)(lo - 1);
}

__global__ void k_run_flags(const uint32_t* __restrict__ leaf_of, uint64_t n, const uint32_t* __restrict__ n_dev,
                            uint32_t* __restrict__ flag) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const uint64_t ne = n_dev ? *n_dev : n;
    flag[e] = e < ne && (e == 0 || leaf_of[e] != leaf_of[e - 1]) ? 1u : 0u;
}

__global__ void k_run_write(const uint32_t* __restrict__ leaf_of, const uint32_t* __restrict__ flag,
                            const uint32_t* __restrict__ ridx, uint64_t n, uint32_t* __restrict__ run_leaf,
                            uint32_t* __restrict__ run_beg) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n || !flag[e]) return;
    run_leaf[ridx[e]] = leaf_of[e];
    run_beg[ridx[e]] = (uint32_t)e;
}

__device__ __forceinline__ uint32_t run_end(const uint32_t* run_beg, uint32_t r, uint32_t R, uint32_t n) {
    return r + 1 < R ? run_beg[r + 1] : n;
}

// A run fits its leaf while the leaf stays within 2 phi entries (the slot
// capacity C is 2 phi rounded up to a multiple of four: only a stride).
__global__ void k_ins_plan(const uint32_t* __restrict__ run_leaf, const uint32_t* __restrict__ run_beg,
                           const uint32_t* __restrict__ ctr, uint64_t m, const DevTree* __restrict__ dt,
                           uint32_t phi, uint32_t* __restrict__ rpieces,
                           uint32_t* __restrict__ rchunks, uint32_t* __restrict__ rsplit, Dirs dirs) {
    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const NodeRec* leaf = dirs.leaf[dt->cur];
    const uint32_t C = 2 * phi;
    const uint32_t R = dt->L ? ctr[1] : 0u;  // an empty index takes the batch as a fresh build
    if (r >= R) {
        rpieces[r] = rchunks[r] = rsplit[r] = 0u;
        return;
    }
    const uint32_t j = run_leaf[r];
    const uint32_t len = run_end(run_beg, (uint32_t)r, R, (uint32_t)m) - run_beg[r];
    const uint32_t t = leaf[j].cnt + len;
    if (t <= C) {
        rpieces[r] = rchunks[r] = rsplit[r] = 0u;
    } else {
        const uint32_t P = (t + phi - 1) / phi;
        rpieces[r] = P;
        rchunks[r] = (t + UPD_CHUNK - 1) / UPD_CHUNK;
        rsplit[r] = 1u;
    }
}

// pieces[run_leaf[r]] = rpieces[r] for the runs whose leaf is re-cut (the
// other leaves keep the one piece the caller filled in).
__global__ void k_ins_pieces(const uint32_t* __restrict__ run_leaf, const uint32_t* __restrict__ ctr, uint64_t m,
                             const uint32_t* __restrict__ rpieces, const uint32_t* __restrict__ rsplit,
                             uint32_t* __restrict__ pieces) {
    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m || r >= ctr[1] || !rsplit[r]) return;
    pieces[run_leaf[r]] = rpieces[r];
}

// Slots for the A = ctr[3] new leaves: the top of the free stack first, then
// fresh ones past the bump pointer (both read from the device state).
__global__ void k_alloc(uint32_t* __restrict__ slot_alloc, const uint32_t* __restrict__ ctr,
                        const uint32_t* __restrict__ free_stack, const DevTree* __restrict__ dt, Caps cap) {
    const uint64_t A = ctr[3], n_free = dt->n_free, slot_top = dt->slot_top;
    for (uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; a < A; a += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t v = a < n_free ? free_stack[n_free - 1 - a] : slot_top + (a - n_free);
        if (v >= cap.slots) {
            atomicOr(cap.err, ERR_CAPACITY);
            slot_alloc[a] = 0;  // never used: the plan check rejects such an update first
            continue;
        }
        slot_alloc[a] = (uint32_t)v;
    }
}

// Untouched leaves move to the other directory buffer when the insert re-cuts
// leaves (ctr[3] > 0); otherwise the directory is updated in place.
__global__ void k_dir_copy(const DevTree* __restrict__ dt, const uint32_t* __restrict__ ctr,
                           const uint32_t* __restrict__ pieces, const uint32_t* __restrict__ newpos, Caps cap) {
    if (ctr[3] == 0) return;  // nothing re-cut: the directory is updated in place
    const uint64_t L = dt->L;
    const uint32_t c = dt->cur;
    const NodeRec* src = cap.dirs.leaf[c];
    const uint64_t* spk = cap.dirs.pkey[c];
    const uint32_t* spi = cap.dirs.pid[c];
    NodeRec* dst = cap.dirs.leaf[1 - c];
    uint64_t* dpk = cap.dirs.pkey[1 - c];
    uint32_t* dpi = cap.dirs.pid[1 - c];
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < L; j += (uint64_t)gridDim.x * blockDim.x) {
    if (pieces[j] != 1u) continue;
    const uint32_t q = newpos[j];
    if (q >= cap.leaves) {
        atomicOr(cap.err, ERR_CAPACITY);
        continue;
    }
    dst[q] = src[j];
    dpk[q] = spk[j];
    dpi[q] = spi[j];
    }
}

template <int D, int CURVE>
__global__ __launch_bounds__(256) void k_ins_append(const uint64_t* __restrict__ bk, const uint32_t* __restrict__ bi,
                                                    const uint32_t* __restrict__ run_leaf,
                                                    const uint32_t* __restrict__ run_beg,
                                                    const uint32_t* __restrict__ ctr, uint64_t m,
                                                    const uint32_t* __restrict__ rsplit,
                                                    const uint32_t* __restrict__ newpos, const DevTree* __restrict__ dt,
                                                    uint32_t* __restrict__ slots, uint32_t C,
                                                    uint32_t* __restrict__ err, Caps cap) {
    // Hilbert keys decode through the curve's table staged in LDS (a lookup
    // per two planes: eleven dependent reads per point)
    __shared__ uint16_t s_h[CURVE ? HilbertFsm<D>::ENTRIES : 1];
    if (CURVE) {
        stage_hilbert<D>(s_h, false);
        __syncthreads();
    }
    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t R = ctr[1];
    if (r >= R || rsplit[r]) return;
    const bool recut = ctr[3] != 0;
    const uint32_t dc = recut ? 1 - dt->cur : dt->cur;
    NodeRec* dleaf = cap.dirs.leaf[dc];
    uint64_t* dpk = cap.dirs.pkey[dc];
    uint32_t* dpi = cap.dirs.pid[dc];
    const uint32_t j = run_leaf[r];
    const uint32_t beg = run_beg[r], end = run_end(run_beg, (uint32_t)r, R, (uint32_t)m);
    const uint32_t q = recut ? newpos[j] : j;  // no re-cut leaves: the directory keeps its order
    if (q >= cap.leaves) {
        atomicOr(err, ERR_CAPACITY);
        return;
    }
    NodeRec rec = dleaf[q];
    if (rec.cnt + (end - beg) > C || rec.slot >= cap.slots) {
        atomicOr(err, ERR_CAPACITY);
        return;
    }
    uint32_t* s = slots + (uint64_t)rec.slot * (D + 1) * C;
    for (uint32_t e = beg; e < end; ++e) {
        uint32_t p[D];
        if (CURVE) hilbert_point_fsm<D>(bk[e], p, s_h);
        else morton_point<D>(bk[e], p);
        const uint32_t o = rec.cnt + (e - beg);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            s[d * C + o] = p[d];
            rec.lo[d] = min(rec.lo[d], p[d]);
            rec.hi[d] = max(rec.hi[d], p[d]);
        }
        s[D * C + o] = bi[e];
    }
    rec.cnt += end - beg;
    dleaf[q] = rec;
    if (j == 0 && pair_less(bk[beg], bi[beg], dpk[q], dpi[q])) {
        dpk[q] = bk[beg];
        dpi[q] = bi[beg];
    }
}

// Merge of a leaf (sorted in LDS) with its sorted run, cut into P balanced
// pieces written to fresh slots. A block handles output chunk c (UPD_CHUNK
// outputs); the LDS arrays belong to the caller's loop over chunks.
template <int D, int CURVE>
__device__ __forceinline__ void ins_split_chunk(
    uint32_t c, uint64_t* s_uk, uint64_t* s_ak, uint32_t* s_ui, uint32_t* s_ai, uint32_t (*s_ap)[64],
    const uint64_t* __restrict__ bk, const uint32_t* __restrict__ bi, const uint32_t* __restrict__ run_leaf,
    const uint32_t* __restrict__ run_beg, const uint32_t* __restrict__ ctr, uint64_t m,
    const uint32_t* __restrict__ chunk_off, const uint32_t* __restrict__ piece_off,
    const uint32_t* __restrict__ newpos, const uint32_t* __restrict__ slot_alloc,
    const NodeRec* __restrict__ sleaf, NodeRec* __restrict__ dleaf, uint64_t* __restrict__ dpk,
    uint32_t* __restrict__ dpi, uint32_t* __restrict__ piece_pos, uint32_t* __restrict__ slots, uint32_t C,
    uint32_t phi, Caps cap) {
    const uint32_t R = ctr[1];
    const uint32_t r = find_owner(chunk_off, R, c);
    const uint32_t j = run_leaf[r];
    const uint32_t beg = run_beg[r], end = run_end(run_beg, r, R, (uint32_t)m);
    const uint32_t b = end - beg;
    const NodeRec rec = sleaf[j];
    const uint32_t a = rec.cnt;
    if (a > 64 || a > C || rec.slot >= cap.slots) {  // uniform over the block
        if (threadIdx.x == 0) atomicOr(cap.err, ERR_CAPACITY);
        return;
    }
    const uint32_t t = a + b;
    const uint32_t P = (t + phi - 1) / phi;
    const uint32_t tid = threadIdx.x;
    const uint32_t* s = slots + (uint64_t)rec.slot * (D + 1) * C;
    uint32_t p[D];
    uint64_t key = 0;
    uint32_t id = 0;
    if (tid < a) {
#pragma unroll
        for (int d = 0; d < D; ++d) p[d] = s[d * C + tid];
        id = s[D * C + tid];
        key = sfc_key_tab<D, CURVE>(p);
        s_uk[tid] = key;
        s_ui[tid] = id;
    }
    __syncthreads();
    if (tid < a) {
        uint32_t rank = 0;
        for (uint32_t x = 0; x < a; ++x) rank += pair_less(s_uk[x], s_ui[x], key, id) ? 1u : 0u;
        s_ak[rank] = key;
        s_ai[rank] = id;
#pragma unroll
        for (int d = 0; d < D; ++d) s_ap[d][rank] = p[d];
    }
    __syncthreads();
    const uint64_t k = (uint64_t)(c - chunk_off[r]) * UPD_CHUNK + tid;
    if (k >= t) return;
    // merge path: i = number of leaf entries among the first k outputs
    uint32_t lo = k > b ? (uint32_t)(k - b) : 0u, hi = (uint32_t)min<uint64_t>(k, a);
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        const uint64_t kb = k - mid;  // index into the run
        const bool take = kb >= b || pair_less(s_ak[mid - 1], s_ai[mid - 1], bk[beg + kb], bi[beg + kb]);
        if (take) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t i = lo;
    const uint64_t kb = k - i;
    bool from_a = i < a && (kb >= b || pair_less(s_ak[i], s_ai[i], bk[beg + kb], bi[beg + kb]));
    if (from_a) {
        key = s_ak[i];
        id = s_ai[i];
#pragma unroll
        for (int d = 0; d < D; ++d) p[d] = s_ap[d][i];
    } else {
        key = bk[beg + kb];
        id = bi[beg + kb];
        sfc_point_tab<D, CURVE>(key, p);
    }
    const uint32_t pc = (uint32_t)(((k + 1) * P - 1) / t);
    const uint32_t p0 = (uint32_t)((uint64_t)pc * t / P), p1 = (uint32_t)((uint64_t)(pc + 1) * t / P);
    const uint32_t off = (uint32_t)k - p0;
    const uint64_t ai = (uint64_t)piece_off[r] + pc;
    const uint64_t qq = (uint64_t)newpos[j] + pc;
    if (ai >= cap.alloc || qq >= cap.leaves || rec.slot >= cap.slots) {
        atomicOr(cap.err, ERR_CAPACITY);
        return;
    }
    const uint32_t slot = slot_alloc[ai];
    if (slot >= cap.slots || off >= C) {
        atomicOr(cap.err, ERR_CAPACITY);
        return;
    }
    uint32_t* o = slots + (uint64_t)slot * (D + 1) * C;
#pragma unroll
    for (int d = 0; d < D; ++d) o[d * C + off] = p[d];
    o[D * C + off] = id;
    if (off == 0) {
        const uint32_t q = (uint32_t)qq;
        dpk[q] = key;
        dpi[q] = id;
        NodeRec nr;
        for (int d = 0; d < 3; ++d) {
            nr.lo[d] = 0xFFFFFFFFu;
            nr.hi[d] = 0u;
        }
        nr.cnt = p1 - p0;
        nr.slot = slot;
        dleaf[q] = nr;
        piece_pos[ai] = q;
    }
}

// Persistent over the output chunks of the re-cut leaves (ctr[4] of them):
// the grid is sized by an upper bound, the count is read on the device.
template <int D, int CURVE>
__global__ __launch_bounds__(UPD_CHUNK) void k_ins_split(
    const uint64_t* __restrict__ bk, const uint32_t* __restrict__ bi, const uint32_t* __restrict__ run_leaf,
    const uint32_t* __restrict__ run_beg, const uint32_t* __restrict__ ctr, uint64_t m,
    const uint32_t* __restrict__ chunk_off, const uint32_t* __restrict__ piece_off,
    const uint32_t* __restrict__ newpos, const uint32_t* __restrict__ slot_alloc, const DevTree* __restrict__ dt,
    uint32_t* __restrict__ piece_pos, uint32_t* __restrict__ slots, uint32_t C, uint32_t phi, Caps cap) {
    __shared__ uint64_t s_uk[64], s_ak[64];
    __shared__ uint32_t s_ui[64], s_ai[64];
    __shared__ uint32_t s_ap[D][64];
    const uint32_t nch = ctr[4];
    const uint32_t c0 = dt->cur;
    for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
        __syncthreads();  // the previous chunk's LDS readers are done
        ins_split_chunk<D, CURVE>(c, s_uk, s_ak, s_ui, s_ai, s_ap, bk, bi, run_leaf, run_beg, ctr, m, chunk_off,
                                  piece_off, newpos, slot_alloc, cap.dirs.leaf[c0], cap.dirs.leaf[1 - c0], cap.dirs.pkey[1 - c0],
                                  cap.dirs.pid[1 - c0], piece_pos, slots, C, phi, cap);
    }
}

// Exact boxes of freshly cut pieces (half-wave per piece; pieces hold <= 32).
// Pieces are written to the directory buffer that is not current yet.
template <int D>
__global__ __launch_bounds__(256) void k_piece_meta(const uint32_t* __restrict__ piece_pos,
                                                    const uint32_t* __restrict__ ctr, const DevTree* __restrict__ dt,
                                                    const uint32_t* __restrict__ slots, uint32_t C, Caps cap) {
    const uint64_t A = ctr[3];
    NodeRec* leaf = cap.dirs.leaf[1 - dt->cur];
    const uint32_t t = threadIdx.x & 31;
    const uint64_t step = ((uint64_t)gridDim.x * blockDim.x) >> 5;
    for (uint64_t a = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 5; a < A; a += step) {
    const uint32_t q = piece_pos[a];
    if (q >= cap.leaves) continue;
    NodeRec rec = leaf[q];
    if (rec.slot >= cap.slots || rec.cnt > C) continue;
    const uint32_t* s = slots + (uint64_t)rec.slot * (D + 1) * C;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        uint32_t lo = 0xFFFFFFFFu, hi = 0u;
        for (uint32_t e = t; e < rec.cnt; e += 32) {
            const uint32_t v = s[d * C + e];
            lo = min(lo, v);
            hi = max(hi, v);
        }
        for (int o = 16; o >= 1; o >>= 1) {
            lo = min(lo, shfl_u32(lo, (int)(lane_id() ^ o)));
            hi = max(hi, shfl_u32(hi, (int)(lane_id() ^ o)));
        }
        rec.lo[d] = lo;
        rec.hi[d] = hi;
    }
    if (D == 2) {
        rec.lo[2] = 0;
        rec.hi[2] = 0;
    }
    if (t == 0) leaf[q] = rec;
    }
}

// The slots of the re-cut leaves go on the free stack above what this
// update took from it.
__global__ void k_ins_free(const uint32_t* __restrict__ run_leaf, const uint32_t* __restrict__ ctr, uint64_t m,
                           const uint32_t* __restrict__ rsplit, const uint32_t* __restrict__ free_off,
                           const DevTree* __restrict__ dt, uint32_t* __restrict__ free_stack, Caps cap) {
    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ctr[1] || !rsplit[r]) return;
    const NodeRec* sleaf = cap.dirs.leaf[dt->cur];
    const uint64_t n_free = dt->n_free, A = ctr[3];
    const uint64_t base = n_free - (A < n_free ? A : n_free);
    const uint64_t x = base + free_off[r];
    if (x >= cap.frees) {
        atomicOr(cap.err, ERR_CAPACITY);
        return;
    }
    free_stack[x] = sleaf[run_leaf[r]].slot;
}

// ------------------------------------------------------------------ delete
// Takes the batch: every id below next_id is claimed by swapping its key in
// the id table for the dead mark, so an id already deleted, and every repeat
// of an id after the first, finds the mark and is dropped. A claimed
// (key, id) is routed to its leaf by the current pivots; the sort key is the
// leaf index, or `marker` (above every leaf index) for a dropped entry, so
// that sorting on the leaf bits alone puts the claimed entries first,
// grouped by leaf. The number claimed is added to ctr[0]. Nothing is claimed
// when ctr[9] holds a rejection.
// The route searches the pivot sample (every PSAMPLE-th pivot, `samp`) first,
// then the PSAMPLE pivots it narrows the leaf to.
__global__ void k_del_take(const uint32_t* __restrict__ ids, uint64_t m, uint64_t* __restrict__ idkey,
                           const DevTree* __restrict__ dt, Dirs dirs, const uint4* __restrict__ samp,
                           uint32_t* __restrict__ ctr, uint64_t marker, uint64_t* __restrict__ lk,
                           uint32_t* __restrict__ li) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t id = PAD_ID;
    uint64_t key = DEAD_KEY;
    if (e < m && ctr[9] == 0) {
        id = ids[e];
        if (id < dt->next_id)
            key = atomicExch(reinterpret_cast<unsigned long long*>(idkey + id), (unsigned long long)DEAD_KEY);
    }
    const bool ok = key != DEAD_KEY;
    uint64_t leaf = marker;
    if (ok) {
        const uint32_t c = dt->cur;
        const uint64_t* pk = dirs.pkey[c];
        const uint32_t* pi = dirs.pid[c];
        const uint64_t L = dt->L, ns = (L + PSAMPLE - 1) / PSAMPLE;
        uint64_t lo = 0, hi = ns;  // first sampled pivot greater than (key, id)
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            const uint4 sv = samp[mid];
            if (!pair_less(key, id, ((uint64_t)sv.y << 32) | sv.x, sv.z)) lo = mid + 1;
            else hi = mid;
        }
        // the first pivot greater than (key, id) is in (PSAMPLE (lo - 1), PSAMPLE lo]
        uint64_t a = lo ? (lo - 1) * PSAMPLE : 0, b = min<uint64_t>(lo ? lo * PSAMPLE : PSAMPLE, L);
        if (b - a == PSAMPLE) {
            // a whole stretch: its PSAMPLE keys in one round of loads (16-byte
            // aligned: a is a multiple of PSAMPLE), counting those below the
            // key; a key equal to a pivot's takes the search below (ids)
            const uint4* pv = reinterpret_cast<const uint4*>(pk + a);
            uint4 v[PSAMPLE / 2];
#pragma unroll
            for (uint32_t u = 0; u < PSAMPLE / 2; ++u) v[u] = pv[u];
            uint32_t nb = 0;
            bool tie = false;
#pragma unroll
            for (uint32_t u = 0; u < PSAMPLE / 2; ++u) {
                const uint64_t k0 = ((uint64_t)v[u].y << 32) | v[u].x, k1 = ((uint64_t)v[u].w << 32) | v[u].z;
                nb += (k0 < key ? 1u : 0u) + (k1 < key ? 1u : 0u);
                tie |= k0 == key || k1 == key;
            }
            if (!tie) {
                a += nb;
                b = a;
            }
        }
        while (a < b) {  // a pivot's id is read only when its key ties
            const uint64_t mid = (a + b) >> 1;
            const uint64_t km = pk[mid];
            const bool below = key < km || (key == km && id < pi[mid]);
            if (!below) a = mid + 1;
            else b = mid;
        }
        leaf = a == 0 ? 0u : a - 1;
    }
    if (e < m) {
        lk[e] = leaf;
        li[e] = id;
    }
    const uint64_t b = ballot(ok);
    if (lane_id() == 0 && b) atomicAdd(ctr, (uint32_t)__popcll(b));
}

// Leaf index of every sorted entry (the low word of its sort key), and the
// number deleted to *ndel.
__global__ void k_del_leaf_of(const uint64_t* __restrict__ sk, uint64_t m, const uint32_t* __restrict__ ctr,
                              uint32_t* __restrict__ leaf_of, uint64_t* __restrict__ ndel) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0 && ndel) *ndel = ctr[0];
    if (e < m) leaf_of[e] = (uint32_t)sk[e];
}

// One wave per run: lane e holds leaf entry e; entries whose id is in the
// run are dropped and the survivors are compacted stably in place.
// Deletes inside one leaf per 16-lane group (four leaves per wave): lane g of
// the group holds entries g, g + 16, g + 32, g + 48 (a slot has at most 64).
// Entries whose id is in the leaf's run are removed and the rest are
// compacted in place, keeping their order; the box is recomputed exactly.
constexpr uint32_t DEL_G = 16;
constexpr int DEL_Q = 4;
// Group reductions on the VALU's cross-lane paths (a group is one 16-lane
// row): two quad swaps, then the half-row and row mirrors. Every lane of the
// row must be active.
template <bool MIN>
__device__ __forceinline__ uint32_t grp_reduce(uint32_t v) {
    static_assert(DEL_G == 16, "a group is one DPP row");
    auto op = [](uint32_t a, uint32_t b) { return MIN ? min(a, b) : max(a, b); };
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm [1, 0, 3, 2]
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm [2, 3, 0, 1]
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    return op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
}
__device__ __forceinline__ uint32_t grp_min(uint32_t v) { return grp_reduce<true>(v); }
__device__ __forceinline__ uint32_t grp_max(uint32_t v) { return grp_reduce<false>(v); }

template <int D>
__global__ __launch_bounds__(256) void k_del_remove(const uint32_t* __restrict__ ci,
                                                    const uint32_t* __restrict__ run_leaf,
                                                    const uint32_t* __restrict__ run_beg,
                                                    const uint32_t* __restrict__ ctr, uint64_t m,
                                                    const DevTree* __restrict__ dt, uint32_t* __restrict__ slots,
                                                    uint32_t C, uint32_t half, uint32_t* __restrict__ under,
                                                    uint32_t* __restrict__ err, Caps cap) {
    __shared__ uint32_t s_under;
    NodeRec* leaf = cap.dirs.leaf[dt->cur];
    if (threadIdx.x == 0) s_under = 0;
    const uint64_t r = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / DEL_G;
    const uint32_t lane = lane_id();
    const uint32_t gl = lane % DEL_G, gbase = lane - gl;  // lane in the group, group's first lane
    const uint32_t R = ctr[1];
    // groups past the last run stay for the wave-wide ballots below
    bool act = r < R;
    const uint32_t V = ctr[0];
    const uint32_t j = act ? run_leaf[r] : 0u;
    const uint32_t beg = act ? run_beg[r] : 0u;
    const uint32_t end = act ? run_end(run_beg, (uint32_t)r, R, V) : 0u;
    NodeRec rec = {};
    if (act) rec = leaf[j];
    if (act && (rec.slot >= cap.slots || rec.cnt > C || rec.cnt > DEL_G * DEL_Q)) {
        if (gl == 0) atomicOr(err, ERR_CAPACITY);
        act = false;
    }
    uint32_t* s = slots + (uint64_t)(act ? rec.slot : 0u) * (D + 1) * C;
    bool on[DEL_Q];
    uint32_t p[DEL_Q][D];
    uint32_t id[DEL_Q];
#pragma unroll
    for (int q = 0; q < DEL_Q; ++q) {
        const uint32_t e = gl + DEL_G * q;
        on[q] = act && e < rec.cnt;
        id[q] = PAD_ID;
#pragma unroll
        for (int d = 0; d < D; ++d) p[q][d] = 0;
        if (on[q]) {
#pragma unroll
            for (int d = 0; d < D; ++d) p[q][d] = s[d * C + e];
            id[q] = s[D * C + e];
        }
    }
    bool del[DEL_Q] = {};
    for (uint32_t x0 = beg; x0 < end; x0 += DEL_G) {  // the run's ids, 16 at a time
        const uint32_t rid = x0 + gl < end ? ci[x0 + gl] : PAD_ID;
        const uint32_t nx = min(DEL_G, end - x0);
        for (uint32_t x = 0; x < nx; ++x) {
            const uint32_t other = shfl_u32(rid, (int)(gbase + x));  // the group's lanes all shuffle
#pragma unroll
            for (int q = 0; q < DEL_Q; ++q) del[q] = del[q] | (on[q] & (other == id[q]));
        }
    }
    // `valid` is always true (stored coordinates are below 2^31) but makes the
    // ballots depend on every loaded coordinate, so all loads of the wave have
    // completed before the in-place stores below are issued.
    uint32_t any = 0;
#pragma unroll
    for (int q = 0; q < DEL_Q; ++q)
#pragma unroll
        for (int d = 0; d < D; ++d) any |= p[q][d];
    const bool valid = any < 0x80000000u;
    const uint64_t gmask = 0xFFFFull << gbase;
    uint32_t kept_before = 0, removed = 0;
    uint32_t pos[DEL_Q];
    bool keep[DEL_Q];
#pragma unroll
    for (int q = 0; q < DEL_Q; ++q) {
        keep[q] = on[q] && !del[q] && valid;
        const uint64_t km = ballot(keep[q]) & gmask;
        removed += (uint32_t)__popcll(ballot(on[q] && del[q]) & gmask);
        pos[q] = kept_before + (uint32_t)__popcll(km & ((1ull << lane) - 1ull));
        kept_before += (uint32_t)__popcll(km);
    }
#pragma unroll
    for (int q = 0; q < DEL_Q; ++q) {
        if (keep[q] && pos[q] != gl + DEL_G * q) {
#pragma unroll
            for (int d = 0; d < D; ++d) s[d * C + pos[q]] = p[q][d];
            s[D * C + pos[q]] = id[q];
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        uint32_t lo = 0xFFFFFFFFu, hi = 0u;
#pragma unroll
        for (int q = 0; q < DEL_Q; ++q) {
            lo = min(lo, keep[q] ? p[q][d] : 0xFFFFFFFFu);
            hi = max(hi, keep[q] ? p[q][d] : 0u);
        }
        rec.lo[d] = grp_min(lo);
        rec.hi[d] = grp_max(hi);
    }
    if (act && gl == 0) {
        if (removed != end - beg) atomicOr(err, ERR_DELETE);
        if (kept_before < half) s_under = 1u;
        rec.cnt = kept_before;
        leaf[j] = rec;
    }
    // one device atomic per workgroup at most, none once the flag is up
    // (every thread reaches the barrier: no thread returns early)
    __syncthreads();
    if (threadIdx.x == 0 && s_under && __hip_atomic_load(under, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
        atomicOr(under, 1u);
}

// Per-leaf counts, and per workgroup 1 + its last leaf holding at least
// `half` entries (0 if none) in bmax[blockIdx.x].
// The arrays span an upper bound Lb of the leaf count: entries past the
// device's L are zero, so the scans over Lb entries see only real leaves.
__global__ __launch_bounds__(256) void k_del_counts(const DevTree* __restrict__ dt, uint64_t Lb, uint32_t half,
                                                    const uint32_t* __restrict__ ctr, uint32_t* __restrict__ cnt,
                                                    uint32_t* __restrict__ bmax, Dirs dirs) {
    __shared__ uint32_t s_w[4];
    if (ctr[8] == 0) return;  // no leaf below the minimum: no regrouping
    const uint64_t L = dt->L;
    const NodeRec* leaf = dirs.leaf[dt->cur];
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t last = 0;
    if (j < L) {
        const uint32_t c = leaf[j].cnt;
        cnt[j] = c;
        if (c >= half) last = (uint32_t)(j + 1);
    } else if (j < Lb) {
        cnt[j] = 0;
    }
    last = wave_max_u32(last);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = last;
    __syncthreads();
    if (threadIdx.x == 0) bmax[blockIdx.x] = max(max(s_w[0], s_w[1]), max(s_w[2], s_w[3]));
}

// ctr[7] = max over the nb per-workgroup values (one workgroup).
__global__ __launch_bounds__(256) void k_del_last_full(const uint32_t* __restrict__ bmax, uint64_t nb,
                                                       uint32_t* __restrict__ ctr) {
    __shared__ uint32_t s_w[4];
    if (ctr[8] == 0) return;
    uint32_t m = 0;
    for (uint64_t i = threadIdx.x; i < nb; i += 256) m = max(m, bmax[i]);
    m = wave_max_u32(m);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) ctr[7] = max(max(s_w[0], s_w[1]), max(s_w[2], s_w[3]));
}

__global__ void k_del_starts(const uint32_t* __restrict__ cnt, uint64_t Lb, uint32_t half,
                             const uint32_t* __restrict__ ctr, const DevTree* __restrict__ dt,
                             uint32_t* __restrict__ start) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Lb || ctr[8] == 0) return;
    start[j] = j < dt->L && (j == 0 || (cnt[j - 1] >= half && j < ctr[7])) ? 1u : 0u;
}

__global__ void k_del_groups(const uint32_t* __restrict__ start, const uint32_t* __restrict__ gidx,
                             const DevTree* __restrict__ dt, const uint32_t* __restrict__ ctr,
                             uint32_t* __restrict__ grp_first) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ctr[8] == 0) return;
    const uint64_t L = dt->L;
    if (j < L && start[j]) grp_first[gidx[j]] = (uint32_t)j;
}

__global__ void k_del_gplan(const uint32_t* __restrict__ grp_first, const uint32_t* __restrict__ ctr, uint64_t Lb,
                            const DevTree* __restrict__ dt, const uint32_t* __restrict__ cum, uint32_t phi,
                            uint32_t* __restrict__ gpieces, uint32_t* __restrict__ gchunks,
                            uint32_t* __restrict__ galloc, uint32_t* __restrict__ gfree,
                            uint32_t* __restrict__ gchanged) {
    if (ctr[8] == 0) return;
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= Lb) return;
    const uint64_t L = dt->L;
    const uint32_t G = ctr[6];
    if (g >= G) {
        gpieces[g] = gchunks[g] = galloc[g] = gfree[g] = gchanged[g] = 0u;
        return;
    }
    const uint32_t f = grp_first[g];
    const uint32_t e = g + 1 < G ? grp_first[g + 1] : (uint32_t)L;
    const uint32_t t = cum[e] - cum[f];
    const bool changed = (e - f) > 1 || t == 0;
    const uint32_t P = changed ? (t + phi - 1) / phi : 1u;
    gpieces[g] = P;
    gchunks[g] = changed ? (t + UPD_CHUNK - 1) / UPD_CHUNK : 0u;
    galloc[g] = changed ? P : 0u;
    gfree[g] = changed ? e - f : 0u;
    gchanged[g] = changed ? 1u : 0u;
}

__global__ void k_del_gcopy(const uint32_t* __restrict__ grp_first, const uint32_t* __restrict__ ctr,
                            const uint32_t* __restrict__ gchanged, const uint32_t* __restrict__ gpos,
                            const DevTree* __restrict__ dt, Caps cap) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ctr[6] || gchanged[g] || ctr[5] == 0) return;
    const uint32_t c = dt->cur;
    const NodeRec* src = cap.dirs.leaf[c];
    const uint64_t* spk = cap.dirs.pkey[c];
    const uint32_t* spi = cap.dirs.pid[c];
    NodeRec* dst = cap.dirs.leaf[1 - c];
    uint64_t* dpk = cap.dirs.pkey[1 - c];
    uint32_t* dpi = cap.dirs.pid[1 - c];
    const uint32_t j = grp_first[g], q = gpos[g];
    if (q >= cap.leaves) {
        atomicOr(cap.err, ERR_CAPACITY);
        return;
    }
    dst[q] = src[j];
    dpk[q] = spk[j];
    dpi[q] = spi[j];
}

// Sort the entries of every leaf of a changed group in place, by (key, id).
template <int D, int CURVE>
__global__ __launch_bounds__(256) void k_sort_leaves(const uint32_t* __restrict__ start,
                                                     const uint32_t* __restrict__ gidx,
                                                     const uint32_t* __restrict__ gchanged,
                                                     const uint32_t* __restrict__ ctr,
                                                     const DevTree* __restrict__ dt, uint32_t* __restrict__ slots,
                                                     uint32_t C, Dirs dirs) {
    const uint32_t lane = lane_id();
    if (ctr[5] == 0) return;  // no regrouping
    const uint64_t L = dt->L;
    const NodeRec* leaf = dirs.leaf[dt->cur];
    const uint64_t step = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t j = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; j < L; j += step) {
    const uint32_t g = gidx[j] + start[j] - 1u;
    if (!gchanged[g]) continue;  // uniform over the wave
    const NodeRec rec = leaf[j];
    if (rec.cnt <= 1 || rec.cnt > 64 || rec.cnt > C) continue;
    uint32_t* s = slots + (uint64_t)rec.slot * (D + 1) * C;
    const bool on = lane < rec.cnt;
    uint32_t p[D];
    uint32_t id = PAD_ID;
    uint64_t key = ~0ull;
    if (on) {
#pragma unroll
        for (int d = 0; d < D; ++d) p[d] = s[d * C + lane];
        id = s[D * C + lane];
        key = sfc_key_tab<D, CURVE>(p);
    }
    uint32_t rank = 0;
    for (uint32_t x = 0; x < rec.cnt; ++x) {
        const uint64_t ok = shfl_u64(key, (int)x);
        const uint32_t oi = shfl_u32(id, (int)x);
        rank += pair_less(ok, oi, key, id) ? 1u : 0u;
    }
    if (on) {
#pragma unroll
        for (int d = 0; d < D; ++d) s[d * C + rank] = p[d];
        s[D * C + rank] = id;
    }
    }
}

// After appends, with leaves kept in total order: one wave per run whose
// leaf took its entries by appending re-sorts that leaf (rank of each entry
// among the leaf's entries by (key, id), keys recomputed from the points).
template <int D, int CURVE>
__global__ __launch_bounds__(256) void k_sort_appended(const uint32_t* __restrict__ run_leaf,
                                                       const uint32_t* __restrict__ ctr, uint64_t m,
                                                       const uint32_t* __restrict__ rsplit,
                                                       const uint32_t* __restrict__ newpos,
                                                       const DevTree* __restrict__ dt, uint32_t* __restrict__ slots,
                                                       uint32_t C, Caps cap) {
    const uint64_t r = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t lane = lane_id();
    if (r >= m || r >= ctr[1] || rsplit[r]) return;  // uniform over the wave
    const bool recut = ctr[3] != 0;
    const NodeRec* leaf = cap.dirs.leaf[recut ? 1 - dt->cur : dt->cur];
    const uint32_t j = run_leaf[r];
    const uint32_t q = recut ? newpos[j] : j;
    if (q >= cap.leaves) return;
    const NodeRec rec = leaf[q];
    if (rec.cnt <= 1 || rec.cnt > 64 || rec.cnt > C || rec.slot >= cap.slots) return;
    uint32_t* s = slots + (uint64_t)rec.slot * (D + 1) * C;
    const bool on = lane < rec.cnt;
    uint32_t p[D];
    uint32_t id = PAD_ID;
    uint64_t key = ~0ull;
    if (on) {
#pragma unroll
        for (int d = 0; d < D; ++d) p[d] = s[d * C + lane];
        id = s[D * C + lane];
        key = sfc_key_tab<D, CURVE>(p);
    }
    uint32_t rank = 0;
    for (uint32_t x = 0; x < rec.cnt; ++x) {  // all reads precede the writes: shuffles only
        const uint64_t ok = shfl_u64(key, (int)x);
        const uint32_t oi = shfl_u32(id, (int)x);
        rank += pair_less(ok, oi, key, id) ? 1u : 0u;
    }
    if (on) {
#pragma unroll
        for (int d = 0; d < D; ++d) s[d * C + rank] = p[d];
        s[D * C + rank] = id;
    }
}

// Concatenate the (sorted) leaves of a changed group and cut into P pieces;
// persistent over the ctr[4] output chunks.
template <int D, int CURVE>
__global__ __launch_bounds__(UPD_CHUNK) void k_del_regroup(
    const uint32_t* __restrict__ grp_first, const uint32_t* __restrict__ ctr,
    const uint32_t* __restrict__ chunk_off, const uint32_t* __restrict__ alloc_off,
    const uint32_t* __restrict__ gpos, const uint32_t* __restrict__ cum, const uint32_t* __restrict__ slot_alloc,
    const DevTree* __restrict__ dt, uint32_t* __restrict__ piece_pos, uint32_t* __restrict__ slots, uint32_t C,
    uint32_t phi, Caps cap) {
    const uint32_t G = ctr[6];
    const uint32_t nch = ctr[4];
    const uint64_t L = dt->L;
    const uint32_t c0 = dt->cur;
    const NodeRec* sleaf = cap.dirs.leaf[c0];
    NodeRec* dleaf = cap.dirs.leaf[1 - c0];
    uint64_t* dpk = cap.dirs.pkey[1 - c0];
    uint32_t* dpi = cap.dirs.pid[1 - c0];
    for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const uint32_t g = find_owner(chunk_off, G, c);
    const uint32_t f = grp_first[g];
    const uint32_t e = g + 1 < G ? grp_first[g + 1] : (uint32_t)L;
    const uint32_t t = cum[e] - cum[f];
    const uint32_t P = (t + phi - 1) / phi;
    const uint64_t k = (uint64_t)(c - chunk_off[g]) * UPD_CHUNK + threadIdx.x;
    if (k >= t) continue;
    const uint32_t gp = cum[f] + (uint32_t)k;
    uint32_t lo = f, hi = e;  // source leaf: last s in [f, e) with cum[s] <= gp
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (cum[mid] <= gp) lo = mid;
        else hi = mid;
    }
    const NodeRec src = sleaf[lo];
    const uint32_t so = gp - cum[lo];
    if (src.slot >= cap.slots || so >= C) {
        atomicOr(cap.err, ERR_CAPACITY);
        continue;
    }
    const uint32_t* s = slots + (uint64_t)src.slot * (D + 1) * C;
    uint32_t p[D];
#pragma unroll
    for (int d = 0; d < D; ++d) p[d] = s[d * C + so];
    const uint32_t id = s[D * C + so];
    const uint32_t pc = (uint32_t)(((k + 1) * P - 1) / t);
    const uint32_t p0 = (uint32_t)((uint64_t)pc * t / P), p1 = (uint32_t)((uint64_t)(pc + 1) * t / P);
    const uint32_t off = (uint32_t)k - p0;
    const uint64_t ai = (uint64_t)alloc_off[g] + pc;
    const uint64_t qq = (uint64_t)gpos[g] + pc;
    if (ai >= cap.alloc || qq >= cap.leaves) {
        atomicOr(cap.err, ERR_CAPACITY);
        continue;
    }
    const uint32_t slot = slot_alloc[ai];
    if (slot >= cap.slots || off >= C) {
        atomicOr(cap.err, ERR_CAPACITY);
        continue;
    }
    uint32_t* o = slots + (uint64_t)slot * (D + 1) * C;
#pragma unroll
    for (int d = 0; d < D; ++d) o[d * C + off] = p[d];
    o[D * C + off] = id;
    if (off == 0) {
        const uint32_t q = (uint32_t)qq;
        dpk[q] = sfc_key_tab<D, CURVE>(p);
        dpi[q] = id;
        NodeRec nr;
        for (int d = 0; d < 3; ++d) {
            nr.lo[d] = 0xFFFFFFFFu;
            nr.hi[d] = 0u;
        }
        nr.cnt = p1 - p0;
        nr.slot = slot;
        dleaf[q] = nr;
        piece_pos[ai] = q;
    }
    }
}

__global__ void k_del_free(const uint32_t* __restrict__ start, const uint32_t* __restrict__ gidx,
                           const uint32_t* __restrict__ gchanged, const uint32_t* __restrict__ grp_first,
                           const uint32_t* __restrict__ free_off, const uint32_t* __restrict__ ctr,
                           const DevTree* __restrict__ dt, uint32_t* __restrict__ free_stack, Caps cap) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= dt->L || ctr[5] == 0) return;
    const NodeRec* sleaf = cap.dirs.leaf[dt->cur];
    const uint64_t n_free = dt->n_free, A = ctr[3];
    const uint64_t base = n_free - (A < n_free ? A : n_free);
    const uint32_t g = gidx[j] + start[j] - 1u;
    if (!gchanged[g]) return;
    const uint64_t x = base + free_off[g] + (j - grp_first[g]);
    if (x >= cap.frees) {
        atomicOr(cap.err, ERR_CAPACITY);
        return;
    }
    free_stack[x] = sleaf[j].slot;
}

}  // namespace

#define PSI_DC(F, ...)                                                    \
    do {                                                                   \
        if (dim == 2 && curve == 0) hipLaunchKernelGGL((F<2, 0>), __VA_ARGS__); \
        else if (dim == 2) hipLaunchKernelGGL((F<2, 1>), __VA_ARGS__);          \
        else if (curve == 0) hipLaunchKernelGGL((F<3, 0>), __VA_ARGS__);        \
        else hipLaunchKernelGGL((F<3, 1>), __VA_ARGS__);                        \
    } while (0)
#define PSI_D(F, ...)                                                     \
    do {                                                                   \
        if (dim == 2) hipLaunchKernelGGL((F<2>), __VA_ARGS__);            \
        else hipLaunchKernelGGL((F<3>), __VA_ARGS__);                     \
    } while (0)

// Grid for a grid-stride loop over at most n items.
inline unsigned stride_blocks(uint64_t n, unsigned per) {
    const unsigned g = blocks_for(n, per);
    return g < 1 ? 1u : (g > 8192 ? 8192u : g);
}

void upd_route(hipStream_t st, const uint64_t* bk, const uint32_t* bi, uint64_t n, const uint32_t* n_dev,
               const DevTree* dt, const Dirs& dirs, uint32_t* leaf_of) {
    if (n) hipLaunchKernelGGL(k_route, dim3(blocks_for(n, 256)), dim3(256), 0, st, bk, bi, n, n_dev, dt, leaf_of, dirs);
}
void upd_runs(hipStream_t st, const uint32_t* leaf_of, uint64_t n, const uint32_t* n_dev, uint32_t* flag,
              uint32_t* ridx, uint32_t* run_leaf, uint32_t* run_beg, uint32_t* R_dev, uint32_t* tmp) {
    if (!n) return;
    hipLaunchKernelGGL(k_run_flags, dim3(blocks_for(n, 256)), dim3(256), 0, st, leaf_of, n, n_dev, flag);
    launch_scan_u32(st, flag, ridx, n, R_dev, tmp);
    hipLaunchKernelGGL(k_run_write, dim3(blocks_for(n, 256)), dim3(256), 0, st, leaf_of, flag, ridx, n, run_leaf, run_beg);
}
void upd_ins_plan(hipStream_t st, const uint32_t* run_leaf, const uint32_t* run_beg, const uint32_t* ctr, uint64_t m,
                  const DevTree* dt, const Dirs& dirs, uint32_t phi, uint32_t* rpieces, uint32_t* rchunks,
                  uint32_t* rsplit) {
    hipLaunchKernelGGL(k_ins_plan, dim3(blocks_for(m, 256)), dim3(256), 0, st, run_leaf, run_beg, ctr, m, dt, phi, rpieces, rchunks, rsplit, dirs);
}
void upd_ins_pieces(hipStream_t st, const uint32_t* run_leaf, const uint32_t* ctr, uint64_t m, const uint32_t* rpieces,
                    const uint32_t* rsplit, uint32_t* pieces) {
    hipLaunchKernelGGL(k_ins_pieces, dim3(blocks_for(m, 256)), dim3(256), 0, st, run_leaf, ctr, m, rpieces, rsplit, pieces);
}
void upd_alloc(hipStream_t st, uint32_t* slot_alloc, uint64_t A_max, const uint32_t* ctr, const uint32_t* free_stack,
               const DevTree* dt, Caps cap) {
    if (A_max) hipLaunchKernelGGL(k_alloc, dim3(stride_blocks(A_max, 256)), dim3(256), 0, st, slot_alloc, ctr, free_stack, dt, cap);
}
void upd_dir_copy(hipStream_t st, const DevTree* dt, const uint32_t* ctr, const uint32_t* pieces,
                  const uint32_t* newpos, uint64_t Lb, Caps cap) {
    if (Lb) hipLaunchKernelGGL(k_dir_copy, dim3(stride_blocks(Lb, 256)), dim3(256), 0, st, dt, ctr, pieces, newpos, cap);
}
void upd_ins_append(hipStream_t st, int dim, int curve, const uint64_t* bk, const uint32_t* bi,
                    const uint32_t* run_leaf, const uint32_t* run_beg, const uint32_t* ctr, uint64_t m,
                    const uint32_t* rsplit, const uint32_t* newpos, const DevTree* dt, uint32_t* slots, uint32_t C,
                    uint32_t* err, Caps cap) {
    PSI_DC(k_ins_append, dim3(blocks_for(m, 256)), dim3(256), 0, st, bk, bi, run_leaf, run_beg, ctr, m, rsplit, newpos, dt, slots, C, err, cap);
}
void upd_sort_appended(hipStream_t st, int dim, int curve, const uint32_t* run_leaf, const uint32_t* ctr, uint64_t m,
                       const uint32_t* rsplit, const uint32_t* newpos, const DevTree* dt, uint32_t* slots,
                       uint32_t C, Caps cap) {
    PSI_DC(k_sort_appended, dim3(blocks_for(m, 4)), dim3(256), 0, st, run_leaf, ctr, m, rsplit, newpos, dt, slots, C, cap);
}
void upd_ins_split(hipStream_t st, int dim, int curve, uint64_t nch_max, const uint64_t* bk, const uint32_t* bi,
                   const uint32_t* run_leaf, const uint32_t* run_beg, const uint32_t* ctr, uint64_t m,
                   const uint32_t* chunk_off, const uint32_t* piece_off, const uint32_t* newpos,
                   const uint32_t* slot_alloc, const DevTree* dt, uint32_t* piece_pos, uint32_t* slots, uint32_t C,
                   uint32_t phi, Caps cap) {
    if (nch_max)
        PSI_DC(k_ins_split, dim3(stride_blocks(nch_max, 1)), dim3(UPD_CHUNK), 0, st, bk, bi, run_leaf, run_beg, ctr, m, chunk_off, piece_off, newpos, slot_alloc, dt, piece_pos, slots, C, phi, cap);
}
void upd_piece_meta(hipStream_t st, int dim, const uint32_t* piece_pos, uint64_t A_max, const uint32_t* ctr,
                    const DevTree* dt, const uint32_t* slots, uint32_t C, Caps cap) {
    if (A_max) PSI_D(k_piece_meta, dim3(stride_blocks(A_max, 8)), dim3(256), 0, st, piece_pos, ctr, dt, slots, C, cap);
}
void upd_ins_free(hipStream_t st, const uint32_t* run_leaf, const uint32_t* ctr, uint64_t m, const uint32_t* rsplit,
                  const uint32_t* free_off, const DevTree* dt, uint32_t* free_stack, Caps cap) {
    hipLaunchKernelGGL(k_ins_free, dim3(blocks_for(m, 256)), dim3(256), 0, st, run_leaf, ctr, m, rsplit, free_off, dt, free_stack, cap);
}

void upd_del_take(hipStream_t st, const uint32_t* ids, uint64_t m, uint64_t* idkey, const DevTree* dt, const Dirs& dirs,
                  const uint4* samp, uint32_t* ctr, uint64_t marker, uint64_t* lk, uint32_t* li) {
    hipLaunchKernelGGL(k_del_take, dim3(blocks_for(m, 256)), dim3(256), 0, st, ids, m, idkey, dt, dirs, samp, ctr, marker, lk, li);
}
void upd_del_leaf_of(hipStream_t st, const uint64_t* sk, uint64_t m, const uint32_t* ctr, uint32_t* leaf_of,
                     uint64_t* ndel) {
    hipLaunchKernelGGL(k_del_leaf_of, dim3(blocks_for(m, 256)), dim3(256), 0, st, sk, m, ctr, leaf_of, ndel);
}
void upd_del_remove(hipStream_t st, int dim, const uint32_t* ci, const uint32_t* run_leaf, const uint32_t* run_beg,
                    const uint32_t* ctr, uint64_t m, const DevTree* dt, uint32_t* slots, uint32_t C, uint32_t phi,
                    uint32_t* under, uint32_t* err, Caps cap) {
    const uint32_t half = (phi + 1) / 2;
    PSI_D(k_del_remove, dim3(blocks_for(m, 256 / DEL_G)), dim3(256), 0, st, ci, run_leaf, run_beg, ctr, m, dt, slots, C, half, under, err, cap);
}
void upd_del_plan(hipStream_t st, const DevTree* dt, const Dirs& dirs, uint64_t Lb, uint32_t phi, uint32_t* ctr, uint32_t* cnt,
                  uint32_t* cum, uint32_t* start, uint32_t* gidx, uint32_t* grp_first, uint32_t* gpieces,
                  uint32_t* gchunks, uint32_t* galloc, uint32_t* gfree, uint32_t* gchanged, uint32_t* gpos,
                  uint32_t* chunk_off, uint32_t* alloc_off, uint32_t* free_off, uint32_t* tmp) {
    const uint32_t half = (phi + 1) / 2;
    const unsigned g = blocks_for(Lb, 256);
    // start[] holds the per-workgroup maxima until k_del_starts fills it
    // every launch below exits at once unless the delete left a leaf below
    // the minimum (ctr[8]); the totals then stay 0 and nothing regroups
    hipLaunchKernelGGL(k_del_counts, dim3(g), dim3(256), 0, st, dt, Lb, half, ctr, cnt, start, dirs);
    hipLaunchKernelGGL(k_del_last_full, dim3(1), dim3(256), 0, st, start, (uint64_t)g, ctr);
    launch_scan_u32(st, cnt, cum, Lb, cum + Lb, tmp, ctr + 8);
    hipLaunchKernelGGL(k_del_starts, dim3(g), dim3(256), 0, st, cnt, Lb, half, ctr, dt, start);
    launch_scan_u32(st, start, gidx, Lb, ctr + 6, tmp, ctr + 8);
    hipLaunchKernelGGL(k_del_groups, dim3(g), dim3(256), 0, st, start, gidx, dt, ctr, grp_first);
    hipLaunchKernelGGL(k_del_gplan, dim3(g), dim3(256), 0, st, grp_first, ctr, Lb, dt, cum, phi, gpieces, gchunks, galloc, gfree, gchanged);
    ScanSet sc{{gpieces, galloc, gchunks, gfree},
               {gpos, alloc_off, chunk_off, free_off},
               {ctr + 2, ctr + 3, ctr + 4, ctr + 5},
               {Lb, Lb, Lb, Lb},
               ctr + 8};
    launch_scan_multi(st, sc, 4, tmp);
}
void upd_del_gcopy(hipStream_t st, const uint32_t* grp_first, const uint32_t* ctr, uint64_t Lb,
                   const uint32_t* gchanged, const uint32_t* gpos, const DevTree* dt, Caps cap) {
    hipLaunchKernelGGL(k_del_gcopy, dim3(blocks_for(Lb, 256)), dim3(256), 0, st, grp_first, ctr, gchanged, gpos, dt, cap);
}
void upd_sort_leaves(hipStream_t st, int dim, int curve, const uint32_t* start, const uint32_t* gidx,
                     const uint32_t* gchanged, const uint32_t* ctr, uint64_t Lb, const DevTree* dt, const Dirs& dirs,
                     uint32_t* slots, uint32_t C) {
    PSI_DC(k_sort_leaves, dim3(stride_blocks(Lb, 4)), dim3(256), 0, st, start, gidx, gchanged, ctr, dt, slots, C, dirs);
}
void upd_del_regroup(hipStream_t st, int dim, int curve, uint64_t nch_max, const uint32_t* grp_first,
                     const uint32_t* ctr, const uint32_t* chunk_off, const uint32_t* alloc_off,
                     const uint32_t* gpos, const uint32_t* cum, const uint32_t* slot_alloc, const DevTree* dt,
                     uint32_t* piece_pos, uint32_t* slots, uint32_t C, uint32_t phi, Caps cap) {
    if (nch_max)
        PSI_DC(k_del_regroup, dim3(stride_blocks(nch_max, 1)), dim3(UPD_CHUNK), 0, st, grp_first, ctr, chunk_off, alloc_off, gpos, cum, slot_alloc, dt, piece_pos, slots, C, phi, cap);
}
void upd_del_free(hipStream_t st, const uint32_t* start, const uint32_t* gidx, const uint32_t* gchanged,
                  const uint32_t* grp_first, const uint32_t* free_off, const uint32_t* ctr, uint64_t Lb,
                  const DevTree* dt, uint32_t* free_stack, Caps cap) {
    hipLaunchKernelGGL(k_del_free, dim3(blocks_for(Lb, 256)), dim3(256), 0, st, start, gidx, gchanged, grp_first, free_off, ctr, dt, free_stack, cap);
}

}  // namespace psi
