// Leaf and node construction from sorted (key, id) pairs, and exports.
//
// Alg. 3 (BuildSorted) cuts the sorted sequence into leaves of at most phi
// points, fetches each leaf's points by id and gives every node the box of
// its children. Here the cut is bottom-up: L = ceil(n/phi) balanced chunks,
// one 32-lane group per leaf. A key is a bijection of its grid point, so the
// point is decoded from the key instead of gathered by id: the fill reads the
// sorted pairs once, in order, and never touches the input coordinates again.
#include "psi_hilbert.h"
#include "psi_kern.h"

namespace psi {

namespace {

inline unsigned blocks_for(uint64_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

// 32-lane group reductions on the VALU's cross-lane paths: two quad swaps,
// the half-row and row mirrors (each lane then holds its 16-lane row's
// result) and a swizzle that exchanges the two rows of the 32-lane group.
// Every lane of the group must be active.
constexpr int DPP_QUAD_SWAP1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int DPP_QUAD_SWAP2 = 0x4E;  // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;
constexpr int SWZ_XOR16 = (16 << 10) | 0x1F;  // bitmask mode: lane ^ 16 inside 32 lanes
template <bool MIN>
__device__ __forceinline__ uint32_t half_reduce(uint32_t v) {
    auto op = [](uint32_t a, uint32_t b) { return MIN ? min(a, b) : max(a, b); };
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, DPP_QUAD_SWAP1, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, DPP_QUAD_SWAP2, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, DPP_HALF_MIRROR, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, DPP_MIRROR, 0xF, 0xF, false));
    return op(v, (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, SWZ_XOR16));
}
__device__ __forceinline__ uint32_t half_min(uint32_t v) { return half_reduce<true>(v); }
__device__ __forceinline__ uint32_t half_max(uint32_t v) { return half_reduce<false>(v); }

template <int D, int CURVE>
__global__ __launch_bounds__(256) void k_build_leaves(const uint64_t* __restrict__ sk,
                                                      const uint32_t* __restrict__ sid, uint64_t n, uint64_t L,
                                                      uint32_t C, uint32_t* __restrict__ slots,
                                                      uint64_t* __restrict__ piv_key, uint32_t* __restrict__ piv_id,
                                                      NodeRec* __restrict__ leafrec, const uint64_t* __restrict__ skip) {
    // skip (may be null): a nonzero word there cancels the fill (an insert
    // into an index that turned out not to be empty)
    if (skip && *skip != 0) return;
    // Hilbert keys decode through the curve's state tables, staged once per
    // workgroup (the grid is sized to the chip; half-waves stride over leaves)
    __shared__ uint16_t s_h[CURVE ? HilbertFsm<D>::ENTRIES : 1];
    if (CURVE) {
        stage_hilbert<D>(s_h, false);
        __syncthreads();
    }
    const uint32_t t = threadIdx.x & 31;
    const int hb = (int)(threadIdx.x & 32);  // first lane of this half-wave
    const uint64_t step = ((uint64_t)gridDim.x * blockDim.x) >> 5;
    const uint64_t j_first = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 5;
    // Lanes 0 and 1 of a half-wave follow the first sorted positions of leaves
    // j and j + 1, floor(j n / L), as quotient q and remainder r; a stride of
    // `step` leaves adds floor(step n / L) and step n mod L, so the loop
    // divides nothing. Past the last leaf the position is clamped to n;
    // positions fit in 32 bits since ids do.
    const uint64_t sq = step * n / L;
    const uint32_t sr = (uint32_t)(step * n % L), Lw = (uint32_t)L;  // L < 2^32
    uint64_t q = 0;
    uint32_t r = 0;
    if (t <= 1) {
        const uint64_t x = (j_first + t) * n;
        q = x / L;
        r = (uint32_t)(x % L);
    }
    // first position and count of the half-wave's next leaf (every lane of
    // the half-wave calls it)
    auto next_leaf = [&](uint32_t& b, uint32_t& cnt) {
        const uint32_t bt = (uint32_t)min<uint64_t>(q, n);
        q += sq;
        r += sr;  // below 2 L: a wrap past 2^32 shows as r < sr
        if (r >= Lw || r < sr) {
            r -= Lw;
            ++q;
        }
        b = shfl_u32(bt, hb);
        cnt = shfl_u32(bt, hb + 1) - b;
    };
    // the pairs of leaf j + step are loaded while leaf j is decoded and
    // written (one stride ahead)
    uint32_t cnt = 0;
    uint64_t key = 0;
    uint32_t id = 0;
    if (j_first < L) {
        uint32_t b = 0;
        next_leaf(b, cnt);
        if (t < cnt) {
            key = sk[(uint64_t)b + t];
            id = sid[(uint64_t)b + t];
        }
    }
    for (uint64_t j = j_first; j < L; j += step) {
        uint32_t b1 = 0, cnt1 = 0;
        uint64_t key1 = 0;
        uint32_t id1 = 0;
        if (j + step < L) {  // uniform over the half-wave
            next_leaf(b1, cnt1);
            if (t < cnt1) {
                key1 = sk[(uint64_t)b1 + t];
                id1 = sid[(uint64_t)b1 + t];
            }
        }
        const bool on = t < cnt;
        uint32_t p[D];
        if (on) {
            if (CURVE) hilbert_point_fsm<D>(key, p, s_h);
            else morton_point<D>(key, p);
            uint32_t* s = slots + j * (uint64_t)(D + 1) * C;
#pragma unroll
            for (int d = 0; d < D; ++d) s[d * C + t] = p[d];
            s[D * C + t] = id;
        } else {
#pragma unroll
            for (int d = 0; d < D; ++d) p[d] = 0;
        }
        NodeRec rec;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            rec.lo[d] = 0xFFFFFFFFu;
            rec.hi[d] = 0u;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            rec.lo[d] = half_min(on ? p[d] : 0xFFFFFFFFu);
            rec.hi[d] = half_max(on ? p[d] : 0u);
        }
        if (t == 0) {
            rec.cnt = cnt;
            rec.slot = (uint32_t)j;
            if (D == 2) { rec.lo[2] = 0; rec.hi[2] = 0; }
            leafrec[j] = rec;
            piv_key[j] = key;
            piv_id[j] = id;
        }
        cnt = cnt1;
        key = key1;
        id = id1;
    }
}

// Node levels u0 + 1 .. u0 + k above the leaves (fewer where the tree is
// lower), one subtree per workgroup: the first level's parents are formed
// from the B^k children read straight from memory (level u0 above the
// leaves: the current directory for u0 = 0; one child per lane, coalesced),
// each further level from the one below held in LDS (count = sum, box =
// per-axis min/max of the non-empty children); every level is written out.
// B^k <= KN_CHILD. s_dyn holds B^(k-1) + B^(k-2) records. Grid-stride over
// the subtrees (the grid is sized from a bound of the leaf count; the
// device state holds the layout).
constexpr uint32_t KN_CHILD = 1024;

// Parent of a group of G lanes (G a power of two >= B): lane g of the group
// brings child g (`on`: it exists) and the group reduces by xor shuffles;
// every lane of the group must take part.
template <int D>
__device__ __forceinline__ NodeRec reduce_group(const NodeRec& x, bool on, uint32_t G) {
    uint32_t cnt = on ? x.cnt : 0u, lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = cnt ? x.lo[d] : 0xFFFFFFFFu;
        hi[d] = cnt ? x.hi[d] : 0u;
    }
    for (uint32_t o = G / 2; o >= 1; o >>= 1) {
        const int src = (int)(lane_id() ^ o);
        cnt += shfl_u32(cnt, src);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = min(lo[d], shfl_u32(lo[d], src));
            hi[d] = max(hi[d], shfl_u32(hi[d], src));
        }
    }
    NodeRec p;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        p.lo[d] = d < D ? lo[d % D] : (cnt ? 0u : 0xFFFFFFFFu);
        p.hi[d] = d < D ? hi[d % D] : 0u;
    }
    p.cnt = cnt;
    p.slot = 0xFFFFFFFFu;
    return p;
}

template <int D>
__global__ __launch_bounds__(256) void k_node_levels(const DevTree* __restrict__ dt, uint32_t u0, uint32_t k,
                                                     NodeRec* __restrict__ inner, uint32_t B, Dirs dirs) {
    extern __shared__ NodeRec s_dyn[];
    const uint32_t h = dt->h;
    if (dt->L == 0 || u0 >= h) return;
    const uint32_t kk = min(k, h - u0);
    uint32_t span = 1;  // B^kk: children of one subtree
    for (uint32_t j = 0; j < kk; ++j) span *= B;
    uint32_t G = 2;
    while (G < B) G <<= 1;
    const uint32_t lc = h - u0;  // the children's level
    const uint64_t n_child = dt->lv[lc].n;
    const NodeRec* child = u0 == 0 ? dirs.leaf[dt->cur] : inner + dt->lv[lc].off;
    const uint64_t roots = (n_child + span - 1) / span;
    for (uint64_t w = blockIdx.x; w < roots; w += gridDim.x) {
        const uint64_t c0 = w * span;
        uint32_t cc = (uint32_t)min<uint64_t>(span, n_child - c0);
        const NodeRec* in = child + c0;
        NodeRec* out = s_dyn;
        NodeRec* spare = s_dyn + span / B;
        uint32_t per = span;  // children per subtree at the current child level
        for (uint32_t j = 1; j <= kk; ++j) {
            per /= B;
            const uint32_t l = lc - j;  // parent level
            const uint64_t p0 = w * per;
            const uint32_t pc = (uint32_t)((cc + B - 1) / B);  // parents in this subtree (one per B children)
            NodeRec* gp = inner + dt->lv[l].off + p0;
            // G lanes per parent (G divides the block, so a group never
            // straddles two passes and the pass count is the block's)
            for (uint32_t b0 = 0; b0 < pc * G; b0 += blockDim.x) {
                const uint32_t idx = b0 + threadIdx.x, x = idx / G, g = idx % G;
                const uint32_t c = x * B + g;
                const bool on = x < pc && g < B && c < cc;
                NodeRec r = {};
                if (on) r = in[c];
                r = reduce_group<D>(r, on, G);
                if (g == 0 && x < pc) {
                    out[x] = r;
                    gp[x] = r;
                }
            }
            __syncthreads();
            NodeRec* t = spare;
            spare = out;
            in = out;
            out = t;
            cc = pc;
        }
    }
}

// Every PSAMPLE-th pivot (key, id) of the current directory as one 16-byte
// record {key low, key high, id, 0}: a table small enough to stay in cache
// for the first steps of routing a key to its leaf.
__global__ void k_pivot_sample(const DevTree* __restrict__ dt, Dirs dirs, uint4* __restrict__ out, uint64_t cap) {
    const uint64_t L = dt->L, ns = min<uint64_t>((L + PSAMPLE - 1) / PSAMPLE, cap);
    const uint32_t c = dt->cur;
    const uint64_t* pk = dirs.pkey[c];
    const uint32_t* pi = dirs.pid[c];
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < ns; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = pk[j * PSAMPLE];
        out[j] = make_uint4((uint32_t)k, (uint32_t)(k >> 32), pi[j * PSAMPLE], 0u);
    }
}

// Packed boxes of the current leaves (leaves = true) or of the inner nodes,
// as many as the device state holds; grid-stride over at most `cap` records.
template <int D>
__global__ void k_pack_tree(const DevTree* __restrict__ dt, bool leaves, const NodeRec* __restrict__ inner,
                            uint4* __restrict__ out, Dirs dirs) {
    const uint64_t n = leaves ? dt->L : dt->n_inner;
    const NodeRec* rec = leaves ? dirs.leaf[dt->cur] : inner;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = packed_box<D>(rec[i]);
}

__global__ void k_leaf_counts(const NodeRec* __restrict__ leaf, uint64_t L, uint32_t* __restrict__ cnt) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < L) cnt[j] = leaf[j].cnt;
}

__global__ void k_widen(const uint32_t* __restrict__ in, uint64_t n, uint64_t* __restrict__ out) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) out[j] = in[j];
}

// One wave per leaf: entries sorted by (key, id) inside the leaf by rank.
template <int D, int CURVE>
__global__ __launch_bounds__(256) void k_export_sorted(TreeView t, const uint64_t* __restrict__ off,
                                                       uint64_t* __restrict__ keys, uint32_t* __restrict__ ids,
                                                       uint32_t* __restrict__ pts) {
    const uint64_t j = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t lane = lane_id();
    if (j >= t.L) return;
    const NodeRec r = t.leaf[j];
    const uint32_t* s = t.slots + (uint64_t)r.slot * (D + 1) * t.C;
    for (uint32_t c0 = 0; c0 < r.cnt; c0 += 64) {
        const uint32_t e = c0 + lane;
        const bool on = e < r.cnt;
        uint32_t p[D];
        uint32_t id = 0;
        uint64_t key = 0;
        if (on) {
#pragma unroll
            for (int d = 0; d < D; ++d) p[d] = s[d * t.C + e];
            id = s[D * t.C + e];
            key = sfc_key_tab<D, CURVE>(p);
        }
        // rank against every entry of the leaf
        uint32_t rank = 0;
        for (uint32_t f0 = 0; f0 < r.cnt; f0 += 64) {
            uint32_t q[D];
            uint32_t fid = 0;
            uint64_t fkey = 0;
            const uint32_t f = f0 + lane;
            if (f < r.cnt) {
#pragma unroll
                for (int d = 0; d < D; ++d) q[d] = s[d * t.C + f];
                fid = s[D * t.C + f];
                fkey = sfc_key_tab<D, CURVE>(q);
            }
            const uint32_t lim = min(64u, r.cnt - f0);
            for (uint32_t x = 0; x < lim; ++x) {
                const uint64_t ok = shfl_u64(fkey, (int)x);
                const uint32_t oi = shfl_u32(fid, (int)x);
                rank += pair_less(ok, oi, key, id) ? 1u : 0u;
            }
        }
        if (on) {
            const uint64_t o = off[j] + rank;
            if (keys) keys[o] = key;
            if (ids) ids[o] = id;
            if (pts) {
#pragma unroll
                for (int d = 0; d < D; ++d) pts[o * D + d] = p[d];
            }
        }
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_export_raw(TreeView t, const uint64_t* __restrict__ off,
                                                    uint32_t* __restrict__ ids, uint32_t* __restrict__ pts) {
    const uint64_t j = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t lane = lane_id();
    if (j >= t.L) return;
    const NodeRec r = t.leaf[j];
    const uint32_t* s = t.slots + (uint64_t)r.slot * (D + 1) * t.C;
    for (uint32_t e = lane; e < r.cnt; e += 64) {
        const uint64_t o = off[j] + e;
        if (ids) ids[o] = s[D * t.C + e];
        if (pts) {
#pragma unroll
            for (int d = 0; d < D; ++d) pts[o * D + d] = s[d * t.C + e];
        }
    }
}

template <int D>
__global__ void k_export_structure(TreeView t, uint64_t n_inner, const uint64_t* __restrict__ pk_src,
                                   const uint32_t* __restrict__ pi_src, uint64_t* __restrict__ piv_key,
                                   uint32_t* __restrict__ piv_id, uint32_t* __restrict__ leaf_cnt,
                                   uint32_t* __restrict__ leaf_lo, uint32_t* __restrict__ leaf_hi,
                                   uint32_t* __restrict__ node_lo, uint32_t* __restrict__ node_hi,
                                   uint64_t* __restrict__ node_cnt) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inner + t.L) return;
    const bool is_leaf = i >= n_inner;
    const NodeRec r = is_leaf ? t.leaf[i - n_inner] : t.inner[i];
    if (node_cnt) node_cnt[i] = r.cnt;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (node_lo) node_lo[i * D + d] = r.lo[d];
        if (node_hi) node_hi[i * D + d] = r.hi[d];
    }
    if (is_leaf) {
        const uint64_t j = i - n_inner;
        if (piv_key) piv_key[j] = pk_src[j];
        if (piv_id) piv_id[j] = pi_src[j];
        if (leaf_cnt) leaf_cnt[j] = r.cnt;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (leaf_lo) leaf_lo[j * D + d] = r.lo[d];
            if (leaf_hi) leaf_hi[j * D + d] = r.hi[d];
        }
    }
}

}  // namespace

void launch_build_leaves(hipStream_t st, int dim, int curve, const uint64_t* sk, const uint32_t* sid,
                         uint64_t n, uint64_t L, uint32_t C, uint32_t* slots, uint64_t* piv_key,
                         uint32_t* piv_id, NodeRec* leafrec, const uint64_t* skip) {
    if (L == 0) return;
    unsigned g = blocks_for(L, 256 / 32);
    if (g > 2048) g = 2048;  // 8 workgroups per CU; half-waves stride over the leaves
#define PSI_BL(D, CV) hipLaunchKernelGGL((k_build_leaves<D, CV>), dim3(g), dim3(256), 0, st, sk, sid, n, L, C, slots, piv_key, piv_id, leafrec, skip)
    if (dim == 2 && curve == 0) PSI_BL(2, 0);
    if (dim == 2 && curve == 1) PSI_BL(2, 1);
    if (dim == 3 && curve == 0) PSI_BL(3, 0);
    if (dim == 3 && curve == 1) PSI_BL(3, 1);
#undef PSI_BL
}

void launch_pack_tree(hipStream_t st, int dim, const DevTree* dt, const Dirs& dirs, bool leaves,
                      const NodeRec* inner, uint4* out, uint64_t cap) {
    if (!cap) return;
    unsigned g = blocks_for(cap, 256);
    if (g > 4096) g = 4096;
    if (dim == 2) hipLaunchKernelGGL(k_pack_tree<2>, dim3(g), dim3(256), 0, st, dt, leaves, inner, out, dirs);
    else hipLaunchKernelGGL(k_pack_tree<3>, dim3(g), dim3(256), 0, st, dt, leaves, inner, out, dirs);
}

void launch_node_levels(hipStream_t st, int dim, const DevTree* dt, const Dirs& dirs, uint64_t L_bound,
                        NodeRec* inner, uint32_t B) {
    uint32_t hb = 0;  // height for L_bound leaves: the device's is at most this
    for (uint64_t n = L_bound; n > 1; ++hb) n = (n + B - 1) / B;
    uint32_t k = 1;  // levels per launch: B^k <= KN_CHILD children staged per workgroup
    for (uint64_t p = (uint64_t)B * B; p <= KN_CHILD; p *= B) ++k;
    for (uint32_t u0 = 0; u0 < hb; u0 += k) {
        const uint32_t kk = std::min(k, hb - u0);
        uint64_t n = L_bound;  // bound of the level u0 + kk node count: the subtrees
        for (uint32_t j = 0; j < u0 + kk; ++j) n = (n + B - 1) / B;
        unsigned g = (unsigned)std::min<uint64_t>(std::max<uint64_t>(n, 1), 8192);
        uint64_t span = 1;
        for (uint32_t j = 0; j < k; ++j) span *= B;
        const size_t lds = (span / B + std::max<uint64_t>(span / B / B, 1)) * sizeof(NodeRec);
        if (dim == 2) hipLaunchKernelGGL(k_node_levels<2>, dim3(g), dim3(256), lds, st, dt, u0, k, inner, B, dirs);
        else hipLaunchKernelGGL(k_node_levels<3>, dim3(g), dim3(256), lds, st, dt, u0, k, inner, B, dirs);
    }
}

void launch_pivot_sample(hipStream_t st, const DevTree* dt, const Dirs& dirs, uint4* out, uint64_t cap) {
    if (!cap) return;
    const unsigned g = (unsigned)std::min<uint64_t>((cap + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pivot_sample, dim3(g), dim3(256), 0, st, dt, dirs, out, cap);
}

void launch_leaf_offsets(hipStream_t st, const NodeRec* leaf, uint64_t L, uint64_t* off, uint64_t* tmp) {
    // tmp: at least 2*L + scan_tmp_words(L) + 2 u32 words (as u64 storage)
    uint32_t* cnt = reinterpret_cast<uint32_t*>(tmp);
    uint32_t* ex = cnt + L;
    uint32_t* sc = ex + L + 1;
    if (L) hipLaunchKernelGGL(k_leaf_counts, dim3(blocks_for(L, 256)), dim3(256), 0, st, leaf, L, cnt);
    launch_scan_u32(st, cnt, ex, L, ex + L, sc);
    hipLaunchKernelGGL(k_widen, dim3(blocks_for(L + 1, 256)), dim3(256), 0, st, ex, L + 1, off);
}

void launch_export_sorted(hipStream_t st, int dim, int curve, const TreeView& t, const uint64_t* off,
                          uint64_t* keys, uint32_t* ids, uint32_t* pts) {
    if (t.L == 0) return;
    const unsigned g = blocks_for(t.L, 256 / 64);
#define PSI_EX(D, CV) hipLaunchKernelGGL((k_export_sorted<D, CV>), dim3(g), dim3(256), 0, st, t, off, keys, ids, pts)
    if (dim == 2 && curve == 0) PSI_EX(2, 0);
    if (dim == 2 && curve == 1) PSI_EX(2, 1);
    if (dim == 3 && curve == 0) PSI_EX(3, 0);
    if (dim == 3 && curve == 1) PSI_EX(3, 1);
#undef PSI_EX
}

void launch_export_raw(hipStream_t st, int dim, const TreeView& t, const uint64_t* off, uint32_t* ids,
                       uint32_t* pts) {
    if (t.L == 0) return;
    const unsigned g = blocks_for(t.L, 256 / 64);
    if (dim == 2) hipLaunchKernelGGL(k_export_raw<2>, dim3(g), dim3(256), 0, st, t, off, ids, pts);
    else hipLaunchKernelGGL(k_export_raw<3>, dim3(g), dim3(256), 0, st, t, off, ids, pts);
}

void launch_export_structure(hipStream_t st, int dim, const TreeView& t, uint64_t n_inner,
                             const uint64_t* piv_key_src, const uint32_t* piv_id_src, uint64_t* piv_key,
                             uint32_t* piv_id, uint32_t* leaf_cnt, uint32_t* leaf_lo, uint32_t* leaf_hi,
                             uint32_t* node_lo, uint32_t* node_hi, uint64_t* node_cnt) {
    const uint64_t tot = n_inner + t.L;
    if (tot == 0) return;
    if (dim == 2)
        hipLaunchKernelGGL(k_export_structure<2>, dim3(blocks_for(tot, 256)), dim3(256), 0, st, t, n_inner, piv_key_src, piv_id_src, piv_key, piv_id, leaf_cnt, leaf_lo, leaf_hi, node_lo, node_hi, node_cnt);
    else
        hipLaunchKernelGGL(k_export_structure<3>, dim3(blocks_for(tot, 256)), dim3(256), 0, st, t, n_inner, piv_key_src, piv_id_src, piv_key, piv_id, leaf_cnt, leaf_lo, leaf_hi, node_lo, node_hi, node_cnt);
}

}  // namespace psi
