// Curve encoding and the LSD radix sort of (key, id) pairs.
//
// Alg. 3 sorts only (code, id) pairs and computes each code when its point is
// first touched. Here the first touch is the histogram kernel: it reads the
// coordinates once, writes the keys (which double as the id -> key table used
// by deletes) and counts the digits of all eight passes. Each pass is then one
// read and one write of the pairs: a tile ranks its pairs with wave ballots,
// learns its global offset by a decoupled look-back over earlier tiles, stages
// the pairs in LDS in digit order and writes them out in digit runs.
#include "psi_hilbert.h"
#include "psi_kern.h"

namespace psi {

namespace {

constexpr int WAVES = SORT_WG / 64;
constexpr uint32_t FLAG_AGG = 1u, FLAG_INC = 2u;
constexpr uint32_t SPIN_LIMIT = 1u << 20;

__device__ __forceinline__ uint64_t pack_status(uint32_t epoch, uint32_t flag, uint32_t v) {
    return ((uint64_t)epoch << 34) | ((uint64_t)flag << 32) | v;
}

__global__ __launch_bounds__(256) void k_hist_pairs(const uint64_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ ids, uint32_t id_base,
                                                    uint64_t n, PassList pl, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[MAX_PASSES][RADIX];
    for (int i = threadIdx.x; i < MAX_PASSES * RADIX; i += blockDim.x) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t k = keys[i];
        const uint32_t id = ids ? ids[i] : id_base + (uint32_t)i;
        for (int p = 0; p < pl.n; ++p) {
            const uint32_t dg = (pl.src[p] ? (uint64_t)id >> pl.shift[p] : k >> pl.shift[p]) & (RADIX - 1);
            atomicAdd(&h[p][dg], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < pl.n * RADIX; i += blockDim.x) {
        const uint32_t v = (&h[0][0])[i];
        if (v) atomicAdd(&hist[i], v);
    }
}

template <int D, int CURVE, bool HIST>
__global__ __launch_bounds__(256) void k_encode_hist(const uint32_t* __restrict__ pts, uint64_t n,
                                                     uint64_t* __restrict__ keys, uint32_t* __restrict__ hist,
                                                     uint32_t* __restrict__ err, int rows, uint32_t shift0,
                                                     uint64_t* __restrict__ kmax) {
    __shared__ uint32_t h[HIST ? 8 : 1][RADIX];
    __shared__ uint64_t s_max[4];
    // Hilbert keys come from the curve's state tables, staged once per
    // workgroup (grid-stride loop below)
    __shared__ uint16_t s_h[CURVE ? HilbertFsm<D>::ENTRIES : 1];
    uint64_t km = 0;
    if (HIST)
        for (int i = threadIdx.x; i < 8 * RADIX; i += blockDim.x) (&h[0][0])[i] = 0;
    if (CURVE) stage_hilbert<D>(s_h, true);
    if (HIST || CURVE) __syncthreads();
    bool bad = false;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t p[D];
#pragma unroll
        for (int d = 0; d < D; ++d) p[d] = pts[i * D + d];
        bad |= !coord_ok<D>(p);
        const uint64_t k = CURVE ? hilbert_key_fsm<D>(p, s_h) : morton_key<D>(p);
        keys[i] = k;
        km = max(km, k);
        if (HIST) {
#pragma unroll
            for (int b = 0; b < 8; ++b)
                if (b < rows) atomicAdd(&h[b][(k >> (shift0 + 8 * b)) & 255u], 1u);
        }
    }
    if (bad) atomicOr(err, ERR_RANGE);
    if (kmax) {  // largest key: one atomic per block
        for (int o = 32; o >= 1; o >>= 1) km = max(km, shfl_u64(km, (int)(lane_id() ^ o)));
        if (lane_id() == 0) s_max[threadIdx.x >> 6] = km;
        __syncthreads();
        if (threadIdx.x == 0)
            atomicMax(reinterpret_cast<unsigned long long*>(kmax),
                      (unsigned long long)max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3])));
    }
    if (HIST) {
        __syncthreads();
        for (int i = threadIdx.x; i < rows * RADIX; i += blockDim.x) {
            const uint32_t v = (&h[0][0])[i];
            if (v) atomicAdd(&hist[i], v);
        }
    }
}

// Keys plus the largest key (as k_encode_hist) and, in the same read of the
// points, the per-chunk counts of the two bucket digits at bits s0 and s1
// that the chunked bucket passes take (the counts k_hist_chunks makes from
// the keys). Each workgroup encodes one contiguous range, so its first-digit
// counts fall in one or two chunks.
template <int D, int CURVE>
__global__ __launch_bounds__(256) void k_encode_chunks(const uint32_t* __restrict__ pts, uint64_t n,
                                                       uint64_t* __restrict__ keys, uint32_t* __restrict__ err,
                                                       uint64_t* __restrict__ kmax, uint32_t s0, uint32_t s1,
                                                       uint64_t T, uint32_t* __restrict__ cnt) {
    __shared__ uint32_t h[2][XCD_CHUNKS][RADIX];
    __shared__ uint64_t s_max[WAVES];
    __shared__ uint16_t s_h[CURVE ? HilbertFsm<D>::ENTRIES : 1];
    for (int i = threadIdx.x; i < 2 * (int)XCD_CHUNKS * RADIX; i += blockDim.x) (&h[0][0][0])[i] = 0;
    if (CURVE) stage_hilbert<D>(s_h, true);
    __syncthreads();
    uint64_t bnd[XCD_CHUNKS];  // first tile of chunks 1 .. 7 (bnd[0] unused)
#pragma unroll
    for (uint32_t x = 0; x < XCD_CHUNKS; ++x) bnd[x] = T * x / XCD_CHUNKS;
    const uint64_t per = ((n + gridDim.x - 1) / gridDim.x + 255) & ~(uint64_t)255;
    const uint64_t b = (uint64_t)blockIdx.x * per, e = min<uint64_t>(b + per, n);
    uint64_t km = 0;
    bool bad = false;
    for (uint64_t i = b + threadIdx.x; i < e; i += 256) {
        uint32_t p[D];
#pragma unroll
        for (int d = 0; d < D; ++d) p[d] = pts[i * D + d];
        bad |= !coord_ok<D>(p);
        const uint64_t k = CURVE ? hilbert_key_fsm<D>(p, s_h) : morton_key<D>(p);
        keys[i] = k;
        km = max(km, k);
        const uint64_t t = i / SORT_TILE;
        uint32_t x = 0;
#pragma unroll
        for (uint32_t y = 1; y < XCD_CHUNKS; ++y) x += t >= bnd[y] ? 1u : 0u;
        const uint32_t d0 = (uint32_t)(k >> s0) & (RADIX - 1), d1 = (uint32_t)(k >> s1) & (RADIX - 1);
        atomicAdd(&h[0][x][d0], 1u);
        atomicAdd(&h[1][d0 >> 5][d1], 1u);
    }
    if (bad) atomicOr(err, ERR_RANGE);
    for (int o = 32; o >= 1; o >>= 1) km = max(km, shfl_u64(km, (int)(lane_id() ^ o)));
    if (lane_id() == 0) s_max[threadIdx.x >> 6] = km;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(reinterpret_cast<unsigned long long*>(kmax),
                  (unsigned long long)max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3])));
    for (int x = threadIdx.x; x < 2 * (int)XCD_CHUNKS * RADIX; x += blockDim.x) {
        const uint32_t v = (&h[0][0][0])[x];
        if (v) atomicAdd(&cnt[x], v);
    }
}

template <int D, int CURVE>
__global__ __launch_bounds__(256) void k_encode_boxes(const uint32_t* __restrict__ boxes, uint64_t n,
                                                      uint64_t* __restrict__ keys) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const uint32_t lo = boxes[i * 2 * D + d], hi = boxes[i * 2 * D + D + d];
        uint32_t v = lo <= hi ? lo + (hi - lo) / 2 : lo;
        v = min(v, D == 2 ? 0x7FFFFFFFu : 0x1FFFFFu);
        c[d] = v;
    }
    keys[i] = sfc_key_tab<D, CURVE>(c);
}

__global__ __launch_bounds__(256) void k_digit_offsets(const uint32_t* __restrict__ hist,
                                                       uint32_t* __restrict__ off) {
    __shared__ uint32_t s_w[WAVES];
    const uint32_t v = hist[blockIdx.x * RADIX + threadIdx.x];
    const uint32_t inc = block_incl_scan256(v, s_w);
    off[blockIdx.x * RADIX + threadIdx.x] = inc - v;
}

// SEG: the pairs form consecutive segments sorted independently (one index
// each); tiles never straddle a segment, digit offsets are per segment and
// the look-back stops at the segment's first tile.
// XCD: the pass is cut into XCD_CHUNKS chunks of consecutive tiles, chunk x
// sorted by the workgroups with blockIdx.x % XCD_CHUNKS == x (which the
// hardware places on one XCD), with its own digit offsets (dig_off row x) and
// a look-back that stops at the chunk's first tile. Consecutive tiles then
// write their digit runs through the same L2, which merges the partial lines.
// Correctness does not depend on the placement.
// LOOP: a workgroup keeps taking tiles (of its chunk, for an XCD pass; below
// *ntiles_dev for a segmented pass) until none is left, so the grid need not
// match the data-dependent tile count; a tile is always processed by the
// workgroup that took it, so every look-back ends. Otherwise a workgroup
// takes one tile (an XCD workgroup finding its chunk exhausted exits).
// shift_dev (may be null): the digit's bit position is shift + *shift_dev.
template <bool IMPLICIT_ID, bool DIGIT_ID, bool SEG, bool XCD = false, bool LOOP = false>
__global__ __launch_bounds__(SORT_WG) void k_onesweep(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ iin, uint32_t id_base,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ iout, uint64_t n, uint32_t shift_arg,
    const uint32_t* __restrict__ dig_off_arg, uint64_t* __restrict__ status, uint32_t* __restrict__ tile_ctr,
    uint32_t epoch, uint32_t* __restrict__ err, SegTiles sg, XcdChunks xc, const uint32_t* __restrict__ shift_dev,
    const uint32_t* __restrict__ ntiles_dev) {
    __shared__ uint64_t s_key[SORT_TILE];
    __shared__ uint32_t s_id[SORT_TILE];
    // running counts per wave, then each wave's first LDS slot per digit; once
    // the tile is staged, row 0 is reused for the global destination of each
    // digit's first slot (52 KB in all: three tiles fit in one CU's LDS)
    __shared__ uint32_t s_wcnt[WAVES][RADIX];
    __shared__ uint32_t s_wsum[WAVES];
    __shared__ uint32_t s_tile, s_nth;

    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const uint32_t lane = lane_id();
    constexpr bool loop = LOOP;
    if (LOOP && SEG && *ntiles_dev == 0) return;  // no tile at all (the usual case of the big-bucket passes)
    const uint32_t shift = shift_arg + (shift_dev ? *shift_dev : 0u);
    for (bool first_round = true;; first_round = false) {
    if (!first_round) {
        if (!loop) break;
        __syncthreads();  // the previous tile's LDS readers are done
    }
    const uint32_t* dig_off = dig_off_arg;
    for (int i = tid; i < WAVES * RADIX; i += SORT_WG) (&s_wcnt[0][0])[i] = 0;
    if (tid == 0) {
        if (XCD) {
            const uint32_t x = blockIdx.x % XCD_CHUNKS;
            const uint32_t t = atomicAdd(tile_ctr + x, 1u);
            s_nth = t;
            s_tile = t < xc.ntiles[x] ? xc.first_tile[x] + t : ~0u;
        } else if (loop) {
            const uint32_t t = atomicAdd(tile_ctr, 1u);
            s_tile = t < *ntiles_dev ? t : ~0u;
        } else {
            s_tile = atomicAdd(tile_ctr, 1u);
        }
    }
    __syncthreads();
    const uint32_t tile = s_tile;
    if (XCD || loop) {
        if (tile == ~0u) break;  // every tile (of the chunk) is taken
    } else if (tile >= gridDim.x) {  // counter not reset: never index past the status array
        if (tid == 0) atomicOr(err, ERR_SPIN);
        return;
    }
    uint64_t tbeg, tend;
    uint32_t first = 0;
    if (XCD) {
        const uint32_t x = blockIdx.x % XCD_CHUNKS;
        tbeg = xc.pos_begin[x] + (uint64_t)s_nth * SORT_TILE;
        tend = min<uint64_t>(tbeg + SORT_TILE, xc.pos_end[x]);
        first = xc.first_tile[x];
        dig_off += (uint64_t)x * RADIX;
    } else if (SEG) {
        const uint32_t sgi = sg.tile_seg[tile];
        tbeg = sg.tile_beg[tile];
        tend = min<uint64_t>(tbeg + SORT_TILE, sg.seg_end[sgi]);
        first = sg.seg_first_tile[sgi];
        dig_off += (uint64_t)sgi * sg.off_stride;
    } else {
        tbeg = (uint64_t)tile * SORT_TILE;
        tend = min<uint64_t>(tbeg + SORT_TILE, n);
    }
    const uint64_t wbase = tbeg + (uint64_t)w * (SORT_IPT * 64);

    uint64_t k[SORT_IPT];
    uint32_t id[SORT_IPT];
    uint32_t rk[SORT_IPT];
#pragma unroll
    for (int i = 0; i < SORT_IPT; ++i) {
        const uint64_t pos = wbase + (uint64_t)i * 64 + lane;
        const bool ok = pos < tend;
        k[i] = ok ? kin[pos] : 0ull;
        id[i] = ok ? (IMPLICIT_ID ? id_base + (uint32_t)pos : iin[pos]) : 0u;
    }
    // Rank inside the wave, item by item (stable: item order = position order).
#pragma unroll
    for (int i = 0; i < SORT_IPT; ++i) {
        const bool ok = wbase + (uint64_t)i * 64 + lane < tend;
        const uint32_t dg = (DIGIT_ID ? (uint64_t)id[i] >> shift : k[i] >> shift) & (RADIX - 1);
        uint64_t peers = ballot(ok);
#pragma unroll
        for (int b = 0; b < RADIX_BITS; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t m = ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t below = count_below(peers);
        const uint32_t base = s_wcnt[w][dg];
        if (ok && below == 0) s_wcnt[w][dg] = base + (uint32_t)__popcll(peers);
        rk[i] = base + below;
    }
    __syncthreads();

    // Thread tid owns digit tid.
    const uint32_t d = tid;
    uint32_t tot = 0;
#pragma unroll
    for (int x = 0; x < WAVES; ++x) {
        const uint32_t c = s_wcnt[x][d];
        s_wcnt[x][d] = tot;
        tot += c;
    }
    uint64_t* my = status + (uint64_t)tile * RADIX + d;
    __hip_atomic_store(my, pack_status(epoch, tile == first ? FLAG_INC : FLAG_AGG, tot), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t loc = block_incl_scan256(tot, s_wsum) - tot;
#pragma unroll
    for (int x = 0; x < WAVES; ++x) s_wcnt[x][d] += loc;

    uint32_t excl = 0;
    if (tile > first) {
        int64_t t = (int64_t)tile - 1;
        uint32_t spins = 0;
        while (t >= (int64_t)first) {
            const uint64_t s = __hip_atomic_load(status + (uint64_t)t * RADIX + d, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t fl = (uint32_t)(s >> 32) & 3u;
            if ((uint32_t)(s >> 34) != epoch || fl == 0) {
                if (++spins > SPIN_LIMIT) {
                    atomicOr(err, ERR_SPIN);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += (uint32_t)s;
            if (fl == FLAG_INC) break;
            --t;
        }
        __hip_atomic_store(my, pack_status(epoch, FLAG_INC, excl + tot), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint32_t my_base = dig_off[d] + excl - loc;
    __syncthreads();

    // Stage in LDS in (digit, position) order.
#pragma unroll
    for (int i = 0; i < SORT_IPT; ++i) {
        const bool ok = wbase + (uint64_t)i * 64 + lane < tend;
        if (ok) {
            const uint32_t dg = (DIGIT_ID ? (uint64_t)id[i] >> shift : k[i] >> shift) & (RADIX - 1);
            const uint32_t lp = s_wcnt[w][dg] + rk[i];
            s_key[lp] = k[i];
            s_id[lp] = id[i];
        }
    }
    __syncthreads();
    uint32_t* s_base = &s_wcnt[0][0];
    s_base[d] = my_base;
    __syncthreads();

    const uint32_t nvalid = (uint32_t)(tend - tbeg);
    for (uint32_t j = tid; j < nvalid; j += SORT_WG) {
        const uint64_t kk = s_key[j];
        const uint32_t ii = s_id[j];
        const uint32_t dg = (DIGIT_ID ? (uint64_t)ii >> shift : kk >> shift) & (RADIX - 1);
        const uint64_t dst = (uint64_t)s_base[dg] + j;
        if (dst < n) {
            kout[dst] = kk;
            iout[dst] = ii;
        } else {
            atomicOr(err, ERR_CAPACITY);
        }
    }
    }
}

// Small batches: every LSD pass of pl inside one workgroup, one launch in
// all. The pairs stay in registers; each pass ranks them (wave ballots, as
// the global passes: stable, item order = position order), writes them to
// their new positions in one LDS copy and reads back the items of the new
// order. 16 waves; wave w owns positions [w * SMALL_PER_WAVE, ...), lane l
// of item i position w * SMALL_PER_WAVE + i * 64 + l.
constexpr int SMALL_WAVES = 16, SMALL_IPT = SORT_SMALL_MAX / (SMALL_WAVES * 64);
constexpr uint32_t SMALL_PER_WAVE = SMALL_IPT * 64;
static_assert(SMALL_IPT * SMALL_WAVES * 64 == SORT_SMALL_MAX, "whole items per thread");
__global__ __launch_bounds__(1024) void k_sort_small(const uint64_t* __restrict__ kin,
                                                     const uint32_t* __restrict__ iin, uint32_t id_base,
                                                     uint32_t n, PassList pl, uint64_t* __restrict__ kout,
                                                     uint32_t* __restrict__ iout) {
    __shared__ uint64_t s_k[SORT_SMALL_MAX];
    __shared__ uint32_t s_i[SORT_SMALL_MAX];
    __shared__ uint32_t s_cnt[SMALL_WAVES][RADIX];
    __shared__ uint32_t s_ws[RADIX / 64];
    const int tid = threadIdx.x, w = tid >> 6;
    const uint32_t lane = lane_id();
    uint64_t k[SMALL_IPT];
    uint32_t id[SMALL_IPT];
#pragma unroll
    for (int i = 0; i < SMALL_IPT; ++i) {
        const uint32_t pos = w * SMALL_PER_WAVE + i * 64 + lane;
        k[i] = pos < n ? kin[pos] : 0ull;
        id[i] = pos < n ? (iin ? iin[pos] : id_base + pos) : 0u;
    }
    for (int p = 0; p < pl.n; ++p) {
        for (int x = tid; x < SMALL_WAVES * RADIX; x += blockDim.x) (&s_cnt[0][0])[x] = 0;
        __syncthreads();
        const uint32_t shift = pl.shift[p];
        const bool by_id = pl.src[p] == 1;
        uint32_t rk[SMALL_IPT];
#pragma unroll
        for (int i = 0; i < SMALL_IPT; ++i) {
            const bool ok = w * SMALL_PER_WAVE + i * 64 + lane < n;
            const uint32_t d = (uint32_t)((by_id ? (uint64_t)id[i] : k[i]) >> shift) & (RADIX - 1);
            uint64_t peers = ballot(ok);
#pragma unroll
            for (int b = 0; b < RADIX_BITS; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = ballot(bit);
                peers &= bit ? m : ~m;
            }
            const uint32_t below = count_below(peers);
            const uint32_t base = s_cnt[w][d];
            if (ok && below == 0) s_cnt[w][d] = base + (uint32_t)__popcll(peers);
            rk[i] = base + below;
        }
        __syncthreads();
        // thread d < 256: its digit's column becomes exclusive over the waves,
        // then every slot gets the digit's start (exclusive prefix over digits)
        uint32_t tot = 0;
        if (tid < RADIX) {
            for (int x = 0; x < SMALL_WAVES; ++x) {
                const uint32_t c = s_cnt[x][tid];
                s_cnt[x][tid] = tot;
                tot += c;
            }
        }
        uint32_t v = tot;  // inclusive scan inside each wave (all lanes take part)
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = shfl_u32(v, (int)lane - o);
            if (lane >= (uint32_t)o) v += t;
        }
        if (tid < RADIX && lane == 63) s_ws[w] = v;
        __syncthreads();
        if (tid < RADIX) {
            uint32_t add = 0;
            for (int i = 0; i < w; ++i) add += s_ws[i];
            const uint32_t excl = v + add - tot;
            for (int x = 0; x < SMALL_WAVES; ++x) s_cnt[x][tid] += excl;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < SMALL_IPT; ++i) {
            if (w * SMALL_PER_WAVE + i * 64 + lane < n) {
                const uint32_t d = (uint32_t)((by_id ? (uint64_t)id[i] : k[i]) >> shift) & (RADIX - 1);
                const uint32_t dst = s_cnt[w][d] + rk[i];
                s_k[dst] = k[i];
                s_i[dst] = id[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < SMALL_IPT; ++i) {
            const uint32_t pos = w * SMALL_PER_WAVE + i * 64 + lane;
            if (pos < n) {
                k[i] = s_k[pos];
                id[i] = s_i[pos];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < SMALL_IPT; ++i) {
        const uint32_t pos = w * SMALL_PER_WAVE + i * 64 + lane;
        if (pos < n) {
            kout[pos] = k[i];
            iout[pos] = id[i];
        }
    }
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_iota_u32(uint32_t* p, uint64_t n, uint32_t base) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = base + (uint32_t)i;
}

// ---- exclusive scan (reduce, scan of tile sums, downsweep) ----
constexpr int SCAN_WG = 256, SCAN_IPT = 8, SCAN_TILE = SCAN_WG * SCAN_IPT;

// Exclusive scans of up to four arrays at once: blockIdx.y picks the array,
// so one set of three launches serves them all. Tile sums of array y live at
// sums[y * stride ...].
__global__ __launch_bounds__(256) void k_scan_reduce(ScanSet s, uint32_t* __restrict__ sums, uint64_t stride) {
    __shared__ uint32_t s_w[WAVES];
    if (s.gate && *s.gate == 0) return;
    const int y = blockIdx.y;
    const uint32_t* __restrict__ in = s.in[y];
    const uint64_t n = s.n[y];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    if (base >= n) return;
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < SCAN_IPT; ++i) {
        const uint64_t p = base + (uint64_t)i * SCAN_WG + threadIdx.x;
        if (p < n) v += in[p];
    }
    v = wave_sum_u32(v);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < WAVES; ++i) t += s_w[i];
        sums[y * stride + blockIdx.x] = t;
    }
}

// One block per array: exclusive scan of its tile sums in place; the array's
// total goes to s.total[y] when that is set.
__global__ __launch_bounds__(256) void k_scan_sums(ScanSet s, uint32_t* __restrict__ sums_all, uint64_t stride) {
    __shared__ uint32_t s_w[WAVES];
    __shared__ uint32_t s_tot;
    if (s.gate && *s.gate == 0) return;
    const int y = blockIdx.x;
    uint32_t* __restrict__ sums = sums_all + y * stride;
    const uint64_t m = (s.n[y] + SCAN_TILE - 1) / SCAN_TILE;
    uint32_t carry = 0;
    for (uint64_t b = 0; b < m; b += SCAN_WG) {
        const uint64_t p = b + threadIdx.x;
        const uint32_t v = p < m ? sums[p] : 0u;
        const uint32_t inc = block_incl_scan256(v, s_w);
        if (p < m) sums[p] = carry + inc - v;
        if (threadIdx.x == SCAN_WG - 1) s_tot = inc;
        __syncthreads();
        carry += s_tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && s.total[y]) *s.total[y] = carry;
}

__global__ __launch_bounds__(256) void k_scan_down(ScanSet s, const uint32_t* __restrict__ sums, uint64_t stride) {
    __shared__ uint32_t s_w[WAVES];
    if (s.gate && *s.gate == 0) return;
    const int y = blockIdx.y;
    const uint32_t* __restrict__ in = s.in[y];
    uint32_t* __restrict__ out = s.out[y];
    const uint64_t n = s.n[y];
    if ((uint64_t)blockIdx.x * SCAN_TILE >= n) return;
    // blocked layout: thread t owns items [t*IPT, t*IPT+IPT) of the tile
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_IPT;
    uint32_t v[SCAN_IPT];
    uint32_t t = 0;
#pragma unroll
    for (int i = 0; i < SCAN_IPT; ++i) {
        v[i] = base + i < n ? in[base + i] : 0u;
        t += v[i];
    }
    const uint32_t inc = block_incl_scan256(t, s_w);
    uint32_t run = sums[y * stride + blockIdx.x] + inc - t;
#pragma unroll
    for (int i = 0; i < SCAN_IPT; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

inline unsigned blocks_for(uint64_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

void launch_hist_pairs(hipStream_t st, const uint64_t* keys, const uint32_t* ids, uint32_t id_base,
                       uint64_t n, const PassList& pl, uint32_t* hist) {
    if (n == 0) return;
    unsigned g = blocks_for(n, 256 * 16);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_hist_pairs, dim3(g), dim3(256), 0, st, keys, ids, id_base, n, pl, hist);
}

void launch_encode_hist(hipStream_t st, int dim, int curve, const uint32_t* pts, uint64_t n, uint64_t* keys,
                        uint32_t* hist, uint32_t* err, int rows, uint32_t shift0) {
    if (n == 0) return;
    unsigned g = blocks_for(n, 256 * 16);
    if (g > 4096) g = 4096;
    if (dim == 2 && curve == 0) hipLaunchKernelGGL((k_encode_hist<2, 0, true>), dim3(g), dim3(256), 0, st, pts, n, keys, hist, err, rows, shift0, nullptr);
    if (dim == 2 && curve == 1) hipLaunchKernelGGL((k_encode_hist<2, 1, true>), dim3(g), dim3(256), 0, st, pts, n, keys, hist, err, rows, shift0, nullptr);
    if (dim == 3 && curve == 0) hipLaunchKernelGGL((k_encode_hist<3, 0, true>), dim3(g), dim3(256), 0, st, pts, n, keys, hist, err, rows, shift0, nullptr);
    if (dim == 3 && curve == 1) hipLaunchKernelGGL((k_encode_hist<3, 1, true>), dim3(g), dim3(256), 0, st, pts, n, keys, hist, err, rows, shift0, nullptr);
}

void launch_encode(hipStream_t st, int dim, int curve, const uint32_t* pts, uint64_t n, uint64_t* keys,
                   uint32_t* err, uint64_t* kmax) {
    if (n == 0) return;
    unsigned g = blocks_for(n, 256 * 4);
    if (g > 8192) g = 8192;
    if (dim == 2 && curve == 0) hipLaunchKernelGGL((k_encode_hist<2, 0, false>), dim3(g), dim3(256), 0, st, pts, n, keys, nullptr, err, 0, 0u, kmax);
    if (dim == 2 && curve == 1) hipLaunchKernelGGL((k_encode_hist<2, 1, false>), dim3(g), dim3(256), 0, st, pts, n, keys, nullptr, err, 0, 0u, kmax);
    if (dim == 3 && curve == 0) hipLaunchKernelGGL((k_encode_hist<3, 0, false>), dim3(g), dim3(256), 0, st, pts, n, keys, nullptr, err, 0, 0u, kmax);
    if (dim == 3 && curve == 1) hipLaunchKernelGGL((k_encode_hist<3, 1, false>), dim3(g), dim3(256), 0, st, pts, n, keys, nullptr, err, 0, 0u, kmax);
}

void launch_encode_chunks(hipStream_t st, int dim, int curve, const uint32_t* pts, uint64_t n, uint64_t* keys,
                          uint32_t* err, uint64_t* kmax, uint32_t s0, uint32_t* cnt) {
    if (n == 0) return;
    unsigned g = blocks_for(n, 256 * 4);
    if (g > 8192) g = 8192;
    const uint64_t T = (n + SORT_TILE - 1) / SORT_TILE;
    const uint32_t s1 = s0 + 8;
    if (dim == 2 && curve == 0) hipLaunchKernelGGL((k_encode_chunks<2, 0>), dim3(g), dim3(256), 0, st, pts, n, keys, err, kmax, s0, s1, T, cnt);
    if (dim == 2 && curve == 1) hipLaunchKernelGGL((k_encode_chunks<2, 1>), dim3(g), dim3(256), 0, st, pts, n, keys, err, kmax, s0, s1, T, cnt);
    if (dim == 3 && curve == 0) hipLaunchKernelGGL((k_encode_chunks<3, 0>), dim3(g), dim3(256), 0, st, pts, n, keys, err, kmax, s0, s1, T, cnt);
    if (dim == 3 && curve == 1) hipLaunchKernelGGL((k_encode_chunks<3, 1>), dim3(g), dim3(256), 0, st, pts, n, keys, err, kmax, s0, s1, T, cnt);
}

void launch_encode_boxes(hipStream_t st, int dim, int curve, const uint32_t* boxes, uint64_t n, uint64_t* keys) {
    if (n == 0) return;
    const unsigned g = blocks_for(n, 256);
    if (dim == 2 && curve == 0) hipLaunchKernelGGL((k_encode_boxes<2, 0>), dim3(g), dim3(256), 0, st, boxes, n, keys);
    if (dim == 2 && curve == 1) hipLaunchKernelGGL((k_encode_boxes<2, 1>), dim3(g), dim3(256), 0, st, boxes, n, keys);
    if (dim == 3 && curve == 0) hipLaunchKernelGGL((k_encode_boxes<3, 0>), dim3(g), dim3(256), 0, st, boxes, n, keys);
    if (dim == 3 && curve == 1) hipLaunchKernelGGL((k_encode_boxes<3, 1>), dim3(g), dim3(256), 0, st, boxes, n, keys);
}

void launch_digit_offsets(hipStream_t st, int npass, const uint32_t* hist, uint32_t* off) {
    hipLaunchKernelGGL(k_digit_offsets, dim3(npass), dim3(256), 0, st, hist, off);
}

void launch_onesweep(hipStream_t st, bool implicit_ids, bool digit_from_id, const uint64_t* kin,
                     const uint32_t* iin, uint32_t id_base, uint64_t* kout, uint32_t* iout, uint64_t n,
                     uint32_t shift, const uint32_t* dig_off, uint64_t* status, uint32_t* tile_ctr,
                     uint32_t epoch, uint32_t* err, const SegTiles* seg, uint64_t seg_tiles,
                     const uint32_t* ntiles_dev) {
    if (n == 0) return;
    SegTiles sg{};
    if (seg) sg = *seg;
    const unsigned g = seg ? (unsigned)seg_tiles : blocks_for(n, SORT_TILE);
    if (g == 0) return;
    const uint32_t* nt = seg ? ntiles_dev : nullptr;
#define PSI_OS(I, Dg, S) hipLaunchKernelGGL((k_onesweep<I, Dg, S>), dim3(g), dim3(SORT_WG), 0, st, kin, iin, id_base, kout, iout, n, shift, dig_off, status, tile_ctr, epoch, err, sg, XcdChunks{}, (const uint32_t*)nullptr, nt)
    if (seg && nt) {
        if (implicit_ids)
            hipLaunchKernelGGL((k_onesweep<true, false, true, false, true>), dim3(g), dim3(SORT_WG), 0, st, kin, iin,
                               id_base, kout, iout, n, shift, dig_off, status, tile_ctr, epoch, err, sg, XcdChunks{},
                               (const uint32_t*)nullptr, nt);
        else
            hipLaunchKernelGGL((k_onesweep<false, false, true, false, true>), dim3(g), dim3(SORT_WG), 0, st, kin, iin,
                               id_base, kout, iout, n, shift, dig_off, status, tile_ctr, epoch, err, sg, XcdChunks{},
                               (const uint32_t*)nullptr, nt);
    } else if (seg) {
        if (implicit_ids) PSI_OS(true, false, true);
        else PSI_OS(false, false, true);
    } else if (implicit_ids && !digit_from_id) PSI_OS(true, false, false);
    else if (implicit_ids && digit_from_id) PSI_OS(true, true, false);
    else if (digit_from_id) PSI_OS(false, true, false);
    else PSI_OS(false, false, false);
#undef PSI_OS
}

void launch_onesweep_xcd(hipStream_t st, bool implicit_ids, const uint64_t* kin, const uint32_t* iin,
                         uint32_t id_base, uint64_t* kout, uint32_t* iout, uint64_t n, uint32_t shift,
                         const uint32_t* dig_off, uint64_t* status, uint32_t* tile_ctr, uint32_t epoch, uint32_t* err,
                         const XcdChunks& xc, uint32_t wg_per_chunk, const uint32_t* shift_dev, bool overflow) {
    if (n == 0 || wg_per_chunk == 0) return;
    // one tile per workgroup; then, for chunks holding more tiles than
    // wg_per_chunk, a small launch whose workgroups take the rest (it finds
    // nothing to do when the chunks are balanced)
    const unsigned g = XCD_CHUNKS * wg_per_chunk;
    const unsigned g2 = XCD_CHUNKS * 32;
    if (implicit_ids) {
        hipLaunchKernelGGL((k_onesweep<true, false, false, true>), dim3(g), dim3(SORT_WG), 0, st, kin, iin, id_base,
                           kout, iout, n, shift, dig_off, status, tile_ctr, epoch, err, SegTiles{}, xc, shift_dev,
                           (const uint32_t*)nullptr);
        if (overflow)
            hipLaunchKernelGGL((k_onesweep<true, false, false, true, true>), dim3(g2), dim3(SORT_WG), 0, st, kin, iin,
                               id_base, kout, iout, n, shift, dig_off, status, tile_ctr, epoch, err, SegTiles{}, xc,
                               shift_dev, (const uint32_t*)nullptr);
    } else {
        hipLaunchKernelGGL((k_onesweep<false, false, false, true>), dim3(g), dim3(SORT_WG), 0, st, kin, iin, id_base,
                           kout, iout, n, shift, dig_off, status, tile_ctr, epoch, err, SegTiles{}, xc, shift_dev,
                           (const uint32_t*)nullptr);
        if (overflow)
            hipLaunchKernelGGL((k_onesweep<false, false, false, true, true>), dim3(g2), dim3(SORT_WG), 0, st, kin, iin,
                               id_base, kout, iout, n, shift, dig_off, status, tile_ctr, epoch, err, SegTiles{}, xc,
                               shift_dev, (const uint32_t*)nullptr);
    }
}

void launch_fill_u32(hipStream_t st, uint32_t* p, uint64_t n, uint32_t v) {
    if (n) hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
}
void launch_iota_u32(hipStream_t st, uint32_t* p, uint64_t n, uint32_t base) {
    if (n) hipLaunchKernelGGL(k_iota_u32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, base);
}

uint64_t scan_tmp_words(uint64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

// Arrays of at most SCAN_SMALL words: one workgroup of 1024 threads scans
// each in one launch (a thread owns 16 consecutive words).
constexpr uint64_t SCAN_SMALL = 1024 * 16;
__global__ __launch_bounds__(1024) void k_scan_small(ScanSet s) {
    __shared__ uint32_t s_w[16];
    if (s.gate && *s.gate == 0) return;
    const int y = blockIdx.x;
    const uint32_t* __restrict__ in = s.in[y];
    uint32_t* __restrict__ out = s.out[y];
    const uint64_t n = s.n[y];
    const uint64_t base = (uint64_t)threadIdx.x * 16;
    uint32_t v[16];
    uint32_t t = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        v[i] = base + i < n ? in[base + i] : 0u;
        t += v[i];
    }
    const uint32_t inc = block_incl_scan256(t, s_w);  // any block of up to 16 waves
    uint32_t run = inc - t;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == blockDim.x - 1 && s.total[y]) *s.total[y] = inc;
}

void launch_scan_multi(hipStream_t st, const ScanSet& s, int k, uint32_t* tmp) {
    ScanSet z = s;
    uint64_t tiles = 0, stride = 0;
    for (int y = k; y < SCAN_MULTI; ++y) z.in[y] = nullptr, z.out[y] = nullptr, z.total[y] = nullptr, z.n[y] = 0;
    bool small = true;
    for (int y = 0; y < k; ++y) small = small && z.n[y] <= SCAN_SMALL;
    if (small) {
        hipLaunchKernelGGL(k_scan_small, dim3(k), dim3(1024), 0, st, z);
        return;
    }
    for (int y = 0; y < k; ++y) {
        tiles = std::max<uint64_t>(tiles, (z.n[y] + SCAN_TILE - 1) / SCAN_TILE);
        stride = std::max<uint64_t>(stride, scan_tmp_words(z.n[y]));
    }
    if (tiles) hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles, k), dim3(SCAN_WG), 0, st, z, tmp, stride);
    hipLaunchKernelGGL(k_scan_sums, dim3(k), dim3(SCAN_WG), 0, st, z, tmp, stride);
    if (tiles) hipLaunchKernelGGL(k_scan_down, dim3((unsigned)tiles, k), dim3(SCAN_WG), 0, st, z, tmp, stride);
}

void launch_sort_small(hipStream_t st, const uint64_t* kin, const uint32_t* iin, uint32_t id_base, uint32_t n,
                       const PassList& pl, uint64_t* kout, uint32_t* iout) {
    if (n) hipLaunchKernelGGL(k_sort_small, dim3(1), dim3(1024), 0, st, kin, iin, id_base, n, pl, kout, iout);
}

void launch_scan_u32(hipStream_t st, const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total,
                     uint32_t* tmp, const uint32_t* gate) {
    if (n == 0 && !gate) {
        if (total) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, total, (uint64_t)1, 0u);
        return;
    }
    ScanSet s{};
    s.gate = gate;
    s.in[0] = in;
    s.out[0] = out;
    s.total[0] = total;
    s.n[0] = n;
    launch_scan_multi(st, s, 1, tmp);
}

}  // namespace psi
