// Many independent indexes built together (batched small indexes): one
// segmented encode, one segmented radix sort (a segment per index), one
// leaf fill and one launch per tree height for the node levels of all
// indexes at once.
#include "psi_hilbert.h"
#include "psi_kern.h"

namespace psi {

namespace {

inline unsigned blocks_for(uint64_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

// largest s in [0, num) with off[s] <= x
__device__ __forceinline__ uint32_t owner_of(const uint32_t* off, uint32_t num, uint64_t x) {
    uint32_t lo = 0, hi = num;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <int D, int CURVE>
__global__ __launch_bounds__(256) void k_encode_hist_seg(const uint32_t* __restrict__ pts, SegTiles sg,
                                                         uint64_t* __restrict__ keys, uint32_t* __restrict__ hist,
                                                         uint32_t* __restrict__ err) {
    __shared__ uint32_t h[8][RADIX];
    for (int i = threadIdx.x; i < 8 * RADIX; i += blockDim.x) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint32_t s = sg.tile_seg[blockIdx.x];
    const uint64_t beg = sg.tile_beg[blockIdx.x];
    const uint64_t end = min<uint64_t>(beg + SORT_TILE, sg.seg_end[s]);
    bool bad = false;
    for (uint64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
        uint32_t p[D];
#pragma unroll
        for (int d = 0; d < D; ++d) p[d] = pts[i * D + d];
        bad |= !coord_ok<D>(p);
        const uint64_t k = sfc_key_tab<D, CURVE>(p);
        keys[i] = k;
#pragma unroll
        for (int b = 0; b < 8; ++b) atomicAdd(&h[b][(k >> (8 * b)) & 255u], 1u);
    }
    if (bad) atomicOr(err, ERR_RANGE);
    __syncthreads();
    uint32_t* hs = hist + (uint64_t)s * 8 * RADIX;
    for (int i = threadIdx.x; i < 8 * RADIX; i += blockDim.x) {
        const uint32_t v = (&h[0][0])[i];
        if (v) atomicAdd(&hs[i], v);
    }
}

// Segments blockIdx.x, + gridDim.x, ... below num (or *num_dev).
__global__ __launch_bounds__(256) void k_seg_digit_offsets(const uint32_t* __restrict__ hist,
                                                           const uint64_t* __restrict__ seg_begin,
                                                           uint32_t* __restrict__ off, uint32_t num,
                                                           const uint32_t* __restrict__ num_dev) {
    __shared__ uint32_t s_w[4];
    const uint32_t ns = num_dev ? *num_dev : num;
    const uint32_t p = blockIdx.y;
    for (uint32_t s = blockIdx.x; s < ns; s += gridDim.x) {
    __syncthreads();
    const uint64_t base = ((uint64_t)s * 8 + p) * RADIX;
    const uint32_t v = hist[base + threadIdx.x];
    const uint32_t lane = lane_id();
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = shfl_u32(x, (int)lane - o);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63) s_w[threadIdx.x >> 6] = x;
    __syncthreads();
    uint32_t add = 0;
    for (uint32_t w = 0; w < (threadIdx.x >> 6); ++w) add += s_w[w];
    off[base + threadIdx.x] = (uint32_t)seg_begin[s] + add + x - v;
    }
}

template <int D, int CURVE>
__global__ __launch_bounds__(256) void k_build_leaves_seg(uint32_t num, uint64_t total, const uint32_t* __restrict__ leaf_off,
                                                          const IdxMeta* __restrict__ meta,
                                                          const uint64_t* __restrict__ sk, const uint32_t* __restrict__ sid,
                                                          uint32_t C, uint32_t* __restrict__ slots,
                                                          uint64_t* __restrict__ piv_key, uint32_t* __restrict__ piv_id,
                                                          NodeRec* __restrict__ leafrec) {
    const uint64_t g = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 5;
    const uint32_t t = threadIdx.x & 31;
    if (g >= total) return;
    const uint32_t s = owner_of(leaf_off, num, g);
    const uint32_t n = meta[s].n, L = meta[s].L, base = meta[s].pt_base;
    const uint64_t j = g - leaf_off[s];
    // one division per lane: lane 0 of the half-wave takes the leaf's first
    // position, lane 1 the next leaf's (below 2^32: n is)
    const uint32_t bt = (uint32_t)((j + (t & 1)) * n / L);
    const int hb = (int)(threadIdx.x & 32);
    const uint32_t b = shfl_u32(bt, hb), cnt = shfl_u32(bt, hb + 1) - b;
    const bool on = t < cnt;
    uint32_t p[D];
    uint64_t key = 0;
    uint32_t id = 0;
    if (on) {
        key = sk[(uint64_t)base + b + t];
        id = sid[(uint64_t)base + b + t] - base;  // local id
        sfc_point_tab<D, CURVE>(key, p);
        uint32_t* sl = slots + g * (uint64_t)(D + 1) * C;
#pragma unroll
        for (int d = 0; d < D; ++d) sl[d * C + t] = p[d];
        sl[D * C + t] = id;
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) p[d] = 0;
    }
    NodeRec r;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        r.lo[d] = d < D ? 0xFFFFFFFFu : 0u;
        r.hi[d] = 0u;
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        uint32_t lo = on ? p[d] : 0xFFFFFFFFu, hi = on ? p[d] : 0u;
        for (int o = 16; o >= 1; o >>= 1) {
            lo = min(lo, shfl_u32(lo, (int)(lane_id() ^ o)));
            hi = max(hi, shfl_u32(hi, (int)(lane_id() ^ o)));
        }
        r.lo[d] = lo;
        r.hi[d] = hi;
    }
    if (t == 0) {
        r.cnt = cnt;
        r.slot = (uint32_t)g;
        leafrec[g] = r;
        piv_key[g] = key;
        piv_id[g] = id;
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_node_step_seg(uint32_t num, uint64_t nparents, uint32_t u,
                                                       const uint32_t* __restrict__ pref,
                                                       const IdxMeta* __restrict__ meta,
                                                       const NodeRec* __restrict__ leafrec,
                                                       NodeRec* __restrict__ inner, uint32_t B) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nparents) return;
    const uint32_t s = owner_of(pref, num, g);
    const IdxMeta& m = meta[s];
    const uint32_t l = m.h - u;  // parent level
    const uint32_t i = (uint32_t)(g - pref[s]);
    const uint32_t nchild = m.lvl_n[l + 1];
    NodeRec r;
    for (int d = 0; d < 3; ++d) {
        r.lo[d] = 0xFFFFFFFFu;
        r.hi[d] = 0u;
    }
    uint32_t cnt = 0;
    const uint32_t c0 = i * B, c1 = min(c0 + B, nchild);
    for (uint32_t c = c0; c < c1; ++c) {
        const NodeRec x = (l + 1 == m.h) ? leafrec[m.leaf_base + c] : inner[m.inner_base + m.lvl_off[l + 1] + c];
        if (x.cnt == 0) continue;
        cnt += x.cnt;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            r.lo[d] = min(r.lo[d], x.lo[d]);
            r.hi[d] = max(r.hi[d], x.hi[d]);
        }
    }
    r.cnt = cnt;
    r.slot = 0xFFFFFFFFu;
    if (D == 2 && cnt) {
        r.lo[2] = 0;
        r.hi[2] = 0;
    }
    inner[m.inner_base + m.lvl_off[l] + i] = r;
}

}  // namespace

void launch_encode_hist_seg(hipStream_t st, int dim, int curve, const uint32_t* pts, uint64_t ntiles,
                            const SegTiles& sg, uint64_t* keys, uint32_t* hist, uint32_t* err) {
    if (!ntiles) return;
    const dim3 g((unsigned)ntiles);
    if (dim == 2 && curve == 0) hipLaunchKernelGGL((k_encode_hist_seg<2, 0>), g, dim3(256), 0, st, pts, sg, keys, hist, err);
    if (dim == 2 && curve == 1) hipLaunchKernelGGL((k_encode_hist_seg<2, 1>), g, dim3(256), 0, st, pts, sg, keys, hist, err);
    if (dim == 3 && curve == 0) hipLaunchKernelGGL((k_encode_hist_seg<3, 0>), g, dim3(256), 0, st, pts, sg, keys, hist, err);
    if (dim == 3 && curve == 1) hipLaunchKernelGGL((k_encode_hist_seg<3, 1>), g, dim3(256), 0, st, pts, sg, keys, hist, err);
}

void launch_seg_digit_offsets(hipStream_t st, uint32_t num, const uint32_t* hist, const uint64_t* seg_begin,
                              uint32_t* off, const uint32_t* num_dev) {
    if (num) {
        const unsigned g = num > 1024 ? 1024u : num;
        hipLaunchKernelGGL(k_seg_digit_offsets, dim3(g, 8), dim3(256), 0, st, hist, seg_begin, off, num, num_dev);
    }
}

void launch_build_leaves_seg(hipStream_t st, int dim, int curve, uint32_t num, uint64_t total_leaves,
                             const uint32_t* leaf_off, const IdxMeta* meta, const uint64_t* sk, const uint32_t* sid,
                             uint32_t C, uint32_t* slots, uint64_t* piv_key, uint32_t* piv_id, NodeRec* leafrec) {
    if (!total_leaves) return;
    const unsigned g = blocks_for(total_leaves, 256 / 32);
#define PSI_BLS(D, CV) hipLaunchKernelGGL((k_build_leaves_seg<D, CV>), dim3(g), dim3(256), 0, st, num, total_leaves, leaf_off, meta, sk, sid, C, slots, piv_key, piv_id, leafrec)
    if (dim == 2 && curve == 0) PSI_BLS(2, 0);
    if (dim == 2 && curve == 1) PSI_BLS(2, 1);
    if (dim == 3 && curve == 0) PSI_BLS(3, 0);
    if (dim == 3 && curve == 1) PSI_BLS(3, 1);
#undef PSI_BLS
}

void launch_node_step_seg(hipStream_t st, int dim, uint32_t num, uint64_t nparents, uint32_t u, const uint32_t* pref,
                          const IdxMeta* meta, const NodeRec* leafrec, NodeRec* inner, uint32_t B) {
    if (!nparents) return;
    const unsigned g = blocks_for(nparents, 256);
    if (dim == 2) hipLaunchKernelGGL(k_node_step_seg<2>, dim3(g), dim3(256), 0, st, num, nparents, u, pref, meta, leafrec, inner, B);
    else hipLaunchKernelGGL(k_node_step_seg<3>, dim3(g), dim3(256), 0, st, num, nparents, u, pref, meta, leafrec, inner, B);
}

}  // namespace psi
