// P-Orth tree (Sec. 3): a 2^D-ary tree whose nodes are the cells of a
// regular grid hierarchy over the coordinate domain [0, 2^W)^D (W = 31 in 2D,
// 21 in 3D). A cell is split at its midpoint on every axis; a cell holding
// more than phi points is an interior node, its non-empty sub-cells are its
// children, and a cell with at most phi points (or a single grid point, which
// cannot be split) is a leaf. That is the tree Alg. 1 returns once it merges
// every subtree of at most phi points into one leaf; it does not depend on
// the skeleton height lambda.
//
// The cells of a level are the runs of equal top D*l bits of the Morton key
// (Sec. 3 notes the construction is a sort on those bits), so after the
// points are sorted by Morton key every cell is a contiguous range and the
// whole tree follows from the sorted keys without moving the points again:
//  * leaf cut: the cell of level l around position i holds more than phi
//    points exactly when some run of phi + 1 consecutive keys containing i
//    agrees on its top l levels, so the level of i's leaf is one more than the
//    largest number of levels shared by keys j and j + phi over the phi + 1
//    windows j in [i - phi, i] (at most W), and a leaf starts at i when keys
//    i - 1 and i differ within that many levels;
//  * nodes in depth-first preorder: the interior nodes that open at leaf t
//    are its ancestors below the deepest level it shares with leaf t - 1, so
//    each leaf knows its own position in preorder and those of the nodes it
//    opens from one prefix sum;
//  * a node's subtree ends at the first leaf whose key leaves the cell (a
//    binary search over the leaves' first keys), which gives the index one
//    past the subtree: traversals need no stack and no parent links.
// Queries follow App. C: a subtree is visited unless its box is farther than
// the current k-th distance (equal distances are still visited, so ties are
// resolved by id exactly).
#include "psi_kern.h"

namespace psi {

namespace {

inline unsigned blocks_for(uint64_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

template <int D> struct OrthBits {
    static constexpr uint32_t W = D == 2 ? 31u : 21u;  // levels below the root
    static constexpr uint32_t KB = D * W;              // key bits in use
};

// Number of leading levels (D-bit groups of the Morton key) on which the
// cells of two keys agree; W when the keys are equal.
template <int D> __device__ __forceinline__ uint32_t common_levels(uint64_t a, uint64_t b) {
    const uint64_t x = (a ^ b) & ((1ull << OrthBits<D>::KB) - 1);
    if (x == 0) return OrthBits<D>::W;
    return ((uint32_t)__builtin_clzll(x) - (64u - OrthBits<D>::KB)) / D;
}

constexpr uint32_t OM_HALO = 32;  // keys loaded beyond each side of a tile (leaf size <= 32)
constexpr uint32_t OM_PER = ORTH_TILE / 256;

template <int D, bool WRITE>
__global__ __launch_bounds__(256) void k_orth_marks(const uint64_t* __restrict__ sk, const uint32_t* __restrict__ sid,
                                                    uint64_t n, uint32_t phi, uint32_t* __restrict__ tile_cnt,
                                                    const uint32_t* __restrict__ tile_off,
                                                    uint32_t* __restrict__ lstart, uint8_t* __restrict__ llev,
                                                    uint64_t* __restrict__ fkey, uint4* __restrict__ pts) {
    __shared__ uint64_t s_k[ORTH_TILE + 2 * OM_HALO];  // key at position base - OM_HALO + x
    __shared__ uint8_t s_cp[ORTH_TILE + OM_HALO];      // 1 + levels shared by keys j and j + phi
    __shared__ uint32_t s_w[4];
    const uint64_t base = (uint64_t)blockIdx.x * ORTH_TILE;
    for (uint32_t x = threadIdx.x; x < ORTH_TILE + 2 * OM_HALO; x += 256) {
        const int64_t g = (int64_t)base - (int64_t)OM_HALO + x;
        s_k[x] = (g >= 0 && (uint64_t)g < n) ? sk[g] : 0ull;
    }
    __syncthreads();
    // j = base - OM_HALO + x; 0 when keys j or j + phi fall outside [0, n)
    for (uint32_t x = threadIdx.x; x < ORTH_TILE + OM_HALO; x += 256) {
        const int64_t j = (int64_t)base - (int64_t)OM_HALO + x;
        uint32_t v = 0;
        if (j >= 0 && (uint64_t)j + phi < n) v = 1u + common_levels<D>(s_k[x], s_k[x + phi]);
        s_cp[x] = (uint8_t)v;
    }
    __syncthreads();
    // positions y = OM_PER * thread .. + OM_PER - 1 of the tile, in order
    uint32_t lvl[OM_PER];
    bool st[OM_PER];
    uint32_t c = 0;
#pragma unroll
    for (uint32_t u = 0; u < OM_PER; ++u) {
        const uint32_t y = threadIdx.x * OM_PER + u;
        const uint64_t i = base + y;
        lvl[u] = 0;
        st[u] = false;
        if (i < n) {
            uint32_t m1 = 0;  // windows j in [i - phi, i]
            for (uint32_t x = y + OM_HALO - phi; x <= y + OM_HALO; ++x) m1 = max(m1, (uint32_t)s_cp[x]);
            const uint32_t l = min(m1, OrthBits<D>::W);
            lvl[u] = l;
            st[u] = i == 0 || common_levels<D>(s_k[y + OM_HALO - 1], s_k[y + OM_HALO]) < l;
            c += st[u] ? 1u : 0u;
        }
    }
    const uint32_t incl = block_incl_scan256(c, s_w);
    if (!WRITE) {
        if (threadIdx.x == 255) tile_cnt[blockIdx.x] = incl;
        return;
    }
    uint32_t leaf = tile_off[blockIdx.x] + incl - c;
#pragma unroll
    for (uint32_t u = 0; u < OM_PER; ++u) {
        if (st[u]) {
            const uint32_t y = threadIdx.x * OM_PER + u;
            lstart[leaf] = (uint32_t)(base + y);
            llev[leaf] = (uint8_t)lvl[u];
            fkey[leaf] = s_k[y + OM_HALO];
            ++leaf;
        }
    }
    // the points in key order, coordinates decoded from the keys
    for (uint32_t y = threadIdx.x; y < ORTH_TILE; y += 256) {
        const uint64_t i = base + y;
        if (i >= n) break;
        uint32_t p[3] = {0u, 0u, 0u};
        morton_point<D>(s_k[y + OM_HALO], p);
        pts[i] = make_uint4(p[0], p[1], D == 3 ? p[2] : 0u, sid[i]);
    }
}

// Interior nodes opened at leaf t: levels [s, lv) with s = 0 for the first
// leaf, else one past the levels it shares with leaf t - 1.
template <int D> __device__ __forceinline__ uint32_t open_from(const uint64_t* fkey, uint32_t t) {
    return t ? common_levels<D>(fkey[t - 1], fkey[t]) + 1u : 0u;
}

template <int D>
__global__ __launch_bounds__(256) void k_orth_counts(const uint8_t* __restrict__ llev, const uint64_t* __restrict__ fkey,
                                                     uint32_t L, uint32_t* __restrict__ cnt1,
                                                     uint32_t* __restrict__ maxlev, uint32_t* __restrict__ err) {
    __shared__ uint32_t s_m[4];
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    uint32_t lv = 0;
    if (t < L) {
        lv = llev[t];
        const uint32_t s = open_from<D>(fkey, t);
        if (s > lv) atomicOr(err, ERR_ORTH);
        cnt1[t] = (s <= lv ? lv - s : 0u) + 1u;
    }
    lv = wave_max_u32(lv);
    if (lane_id() == 0) s_m[threadIdx.x >> 6] = lv;
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(maxlev, max(max(s_m[0], s_m[1]), max(s_m[2], s_m[3])));
}

template <int D>
__global__ __launch_bounds__(256) void k_orth_nodes(const uint8_t* __restrict__ llev, const uint64_t* __restrict__ fkey,
                                                    const uint32_t* __restrict__ lstart,
                                                    const uint32_t* __restrict__ base, uint32_t L, uint32_t n,
                                                    uint64_t N, const uint4* __restrict__ pts,
                                                    OrthNode* __restrict__ node, uint8_t* __restrict__ lev) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= L) return;
    const uint32_t lv = llev[t];
    const uint64_t key = fkey[t];
    const uint32_t s = open_from<D>(fkey, t);
    const uint64_t b = base[t];
    const uint32_t pb = lstart[t], pe = t + 1 < L ? lstart[t + 1] : n;
    for (uint32_t l = s; l < lv; ++l) {
        const uint32_t sh = OrthBits<D>::KB - l * D;
        const uint64_t cell = key >> sh;
        uint32_t lo = t + 1, hi = L;  // first later leaf outside the cell
        while (lo < hi) {
            const uint32_t mid = lo + ((hi - lo) >> 1);
            if ((fkey[mid] >> sh) == cell) lo = mid + 1;
            else hi = mid;
        }
        OrthNode r;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            r.lo[d] = 0xFFFFFFFFu;
            r.hi[d] = 0u;
        }
        r.a = lo < L ? base[lo] : (uint32_t)N;
        r.b = (lo < L ? lstart[lo] : n) - pb;
        node[b + (l - s)] = r;
        lev[b + (l - s)] = (uint8_t)l;
    }
    OrthNode r;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        r.lo[d] = d < D ? 0xFFFFFFFFu : 0u;
        r.hi[d] = 0u;
    }
    for (uint32_t x = pb; x < pe; ++x) {
        const uint4 P = pts[x];
        const uint32_t p[3] = {P.x, P.y, P.z};
#pragma unroll
        for (int d = 0; d < D; ++d) {
            r.lo[d] = min(r.lo[d], p[d]);
            r.hi[d] = max(r.hi[d], p[d]);
        }
    }
    r.a = pb;
    r.b = (pe - pb) | ORTH_LEAF;
    const uint64_t v = b + (s <= lv ? lv - s : 0u);
    node[v] = r;
    lev[v] = 0xFF;
}

template <int D>
__global__ __launch_bounds__(256) void k_orth_boxes(uint32_t level, uint64_t N, const uint8_t* __restrict__ lev,
                                                    OrthNode* __restrict__ node) {
    const uint64_t v = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= N || lev[v] != level) return;
    const uint64_t end = min<uint64_t>(node[v].a, N);
    uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
    if (D == 2) lo[2] = 0u;
    uint64_t c = v + 1;
    while (c < end) {  // the children: first child v + 1, then each one's end
        const OrthNode r = node[c];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = min(lo[d], r.lo[d]);
            hi[d] = max(hi[d], r.hi[d]);
        }
        const uint64_t nx = (r.b & ORTH_LEAF) ? c + 1 : (uint64_t)r.a;
        c = nx > c ? nx : c + 1;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        node[v].lo[d] = lo[d];
        node[v].hi[d] = hi[d];
    }
}

// ------------------------------------------------------------------ queries
template <int D> __device__ __forceinline__ uint64_t orth_box_dist(const uint32_t* q, const OrthNode& r) {
    uint64_t s = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const uint32_t x = q[d] < r.lo[d] ? r.lo[d] - q[d] : (q[d] > r.hi[d] ? q[d] - r.hi[d] : 0u);
        s += (uint64_t)x * x;
    }
    return s;
}

template <int D, int K>
__device__ __forceinline__ void orth_scan(const uint4* __restrict__ pts, uint32_t b, uint32_t e, const uint32_t* q,
                                          uint64_t (&bd)[K], uint32_t (&bi)[K]) {
    for (uint32_t x = b; x < e; ++x) {
        const uint4 P = pts[x];
        const uint32_t p[3] = {P.x, P.y, P.z};
        const uint64_t d = pt_dist<D>(q, p);
        if (d <= bd[K - 1] && pair_less(d, P.w, bd[K - 1], bi[K - 1])) topk_insert<K>(bd, bi, d, P.w);
    }
}

// Lane per query. The leaf holding the query's own Morton position and its
// two neighbours in key order are scanned first (one contiguous run of
// points) to start with a small k-th distance; the preorder walk then skips
// them.
template <int D, int K>
__global__ __launch_bounds__(256) void k_orth_knn(OrthView t, const uint32_t* __restrict__ qp,
                                                  const uint64_t* __restrict__ qkeys, uint64_t nq,
                                                  const uint32_t* __restrict__ order, uint32_t* __restrict__ out_ids,
                                                  uint64_t* __restrict__ out_d2) {
    const uint64_t tq = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tq >= nq) return;
    const uint64_t qi = order ? order[tq] : tq;
    uint32_t q[D];
#pragma unroll
    for (int d = 0; d < D; ++d) q[d] = qp[qi * D + d];
    uint64_t bd[K];
    uint32_t bi[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        bd[j] = PAD_D2;
        bi[j] = PAD_ID;
    }
    if (t.N > 0 && t.L > 0) {
        const uint64_t key = qkeys[qi];
        uint32_t lo = 0, hi = t.L;
        while (lo < hi) {
            const uint32_t mid = lo + ((hi - lo) >> 1);
            if (t.fkey[mid] <= key) lo = mid + 1;
            else hi = mid;
        }
        const uint32_t j = lo ? lo - 1 : 0u;
        const uint32_t ja = j ? j - 1 : 0u, jb = min(j + 1, t.L - 1);
        const uint32_t p0 = t.lstart[ja], p1 = jb + 1 < t.L ? t.lstart[jb + 1] : t.n;
        orth_scan<D, K>(t.pts, p0, p1, q, bd, bi);
        uint64_t v = 0;
        while (v < t.N) {
            const OrthNode r = t.node[v];
            const bool leaf = (r.b & ORTH_LEAF) != 0;
            if (orth_box_dist<D>(q, r) <= bd[K - 1]) {
                if (leaf && (r.a < p0 || r.a >= p1)) orth_scan<D, K>(t.pts, r.a, r.a + (r.b & ~ORTH_LEAF), q, bd, bi);
                ++v;
            } else {
                v = leaf ? v + 1 : max<uint64_t>(r.a, v + 1);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        out_ids[qi * K + j] = bi[j];
        out_d2[qi * K + j] = bd[j];
    }
}

// Lane per box; REPORT writes the ids in preorder to out[offsets[b] ..
// offsets[b + 1]).
template <int D, bool REPORT>
__global__ __launch_bounds__(256) void k_orth_range(OrthView t, const uint32_t* __restrict__ boxes, uint64_t nb,
                                                    const uint32_t* __restrict__ order, uint64_t* __restrict__ counts,
                                                    const uint64_t* __restrict__ offsets, uint32_t* __restrict__ out) {
    const uint64_t bx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (bx >= nb) return;
    const uint64_t b = order ? order[bx] : bx;
    uint32_t lo[D], hi[D];
    bool empty = false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = boxes[b * 2 * D + d];
        hi[d] = boxes[b * 2 * D + D + d];
        empty = empty || lo[d] > hi[d];
    }
    uint64_t cnt = 0, o = 0, lim = 0;
    if (REPORT) {
        o = offsets[b];
        lim = offsets[b + 1];
    }
    uint64_t v = empty ? t.N : 0;
    while (v < t.N) {
        const OrthNode r = t.node[v];
        const bool leaf = (r.b & ORTH_LEAF) != 0;
        const uint32_t c = r.b & ~ORTH_LEAF;
        const uint64_t next = leaf ? v + 1 : max<uint64_t>(r.a, v + 1);
        bool inside = true, apart = false;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            apart = apart || r.hi[d] < lo[d] || r.lo[d] > hi[d];
            inside = inside && lo[d] <= r.lo[d] && r.hi[d] <= hi[d];
        }
        if (apart) {
            v = next;
        } else if (inside) {
            if (!REPORT) {
                cnt += c;
            } else {
                uint64_t u = v;  // the subtree's points start at its first leaf's
                while (u < t.N && !(t.node[u].b & ORTH_LEAF)) ++u;
                const uint32_t pb = u < t.N ? t.node[u].a : 0u;
                for (uint32_t e = 0; e < c && o < lim; ++e) out[o++] = t.pts[pb + e].w;
            }
            v = next;
        } else if (leaf) {
            for (uint32_t x = r.a; x < r.a + c; ++x) {
                const uint4 P = t.pts[x];
                const uint32_t p[3] = {P.x, P.y, P.z};
                bool in = true;
#pragma unroll
                for (int d = 0; d < D; ++d) in = in && lo[d] <= p[d] && p[d] <= hi[d];
                if (in) {
                    if (!REPORT) ++cnt;
                    else if (o < lim) out[o++] = P.w;
                }
            }
            v = next;
        } else {
            ++v;
        }
    }
    if (!REPORT) counts[b] = cnt;
}

}  // namespace

void launch_orth_marks(hipStream_t st, int dim, bool write, const uint64_t* sk, const uint32_t* sid, uint64_t n,
                       uint32_t phi, uint32_t* tile_cnt, const uint32_t* tile_off, uint32_t* lstart, uint8_t* llev,
                       uint64_t* fkey, uint4* pts) {
    if (n == 0) return;
    const dim3 g(blocks_for(n, ORTH_TILE));
#define PSI_OM(D, WR) hipLaunchKernelGGL((k_orth_marks<D, WR>), g, dim3(256), 0, st, sk, sid, n, phi, tile_cnt, tile_off, lstart, llev, fkey, pts)
    if (dim == 2) {
        if (write) PSI_OM(2, true);
        else PSI_OM(2, false);
    } else {
        if (write) PSI_OM(3, true);
        else PSI_OM(3, false);
    }
#undef PSI_OM
}

void launch_orth_counts(hipStream_t st, int dim, const uint8_t* llev, const uint64_t* fkey, uint32_t L,
                        uint32_t* cnt1, uint32_t* maxlev, uint32_t* err) {
    if (L == 0) return;
    const dim3 g(blocks_for(L, 256));
    if (dim == 2) hipLaunchKernelGGL((k_orth_counts<2>), g, dim3(256), 0, st, llev, fkey, L, cnt1, maxlev, err);
    else hipLaunchKernelGGL((k_orth_counts<3>), g, dim3(256), 0, st, llev, fkey, L, cnt1, maxlev, err);
}

void launch_orth_nodes(hipStream_t st, int dim, const uint8_t* llev, const uint64_t* fkey, const uint32_t* lstart,
                       const uint32_t* base, uint32_t L, uint32_t n, uint64_t N, const uint4* pts, OrthNode* node,
                       uint8_t* lev) {
    if (L == 0) return;
    const dim3 g(blocks_for(L, 256));
    if (dim == 2) hipLaunchKernelGGL((k_orth_nodes<2>), g, dim3(256), 0, st, llev, fkey, lstart, base, L, n, N, pts, node, lev);
    else hipLaunchKernelGGL((k_orth_nodes<3>), g, dim3(256), 0, st, llev, fkey, lstart, base, L, n, N, pts, node, lev);
}

void launch_orth_boxes(hipStream_t st, int dim, uint32_t level, uint64_t N, const uint8_t* lev, OrthNode* node) {
    if (N == 0) return;
    const dim3 g(blocks_for(N, 256));
    if (dim == 2) hipLaunchKernelGGL((k_orth_boxes<2>), g, dim3(256), 0, st, level, N, lev, node);
    else hipLaunchKernelGGL((k_orth_boxes<3>), g, dim3(256), 0, st, level, N, lev, node);
}

void launch_orth_knn(hipStream_t st, int dim, const OrthView& t, const uint32_t* q, const uint64_t* qkeys,
                     uint64_t nq, const uint32_t* order, uint32_t k, uint32_t* ids, uint64_t* d2) {
    if (nq == 0) return;
    const dim3 g(blocks_for(nq, 256));
#define PSI_OK_(D, K) hipLaunchKernelGGL((k_orth_knn<D, K>), g, dim3(256), 0, st, t, q, qkeys, nq, order, ids, d2)
#define PSI_OK_ALL(D)                                                                                    \
    switch (k) {                                                                                         \
        case 1: PSI_OK_(D, 1); break;   case 2: PSI_OK_(D, 2); break;   case 3: PSI_OK_(D, 3); break;    \
        case 4: PSI_OK_(D, 4); break;   case 5: PSI_OK_(D, 5); break;   case 6: PSI_OK_(D, 6); break;    \
        case 7: PSI_OK_(D, 7); break;   case 8: PSI_OK_(D, 8); break;   case 9: PSI_OK_(D, 9); break;    \
        case 10: PSI_OK_(D, 10); break; case 11: PSI_OK_(D, 11); break; case 12: PSI_OK_(D, 12); break;  \
        case 13: PSI_OK_(D, 13); break; case 14: PSI_OK_(D, 14); break; case 15: PSI_OK_(D, 15); break;  \
        case 16: PSI_OK_(D, 16); break; default: break;                                                  \
    }
    if (dim == 2) { PSI_OK_ALL(2) } else { PSI_OK_ALL(3) }
#undef PSI_OK_ALL
#undef PSI_OK_
}

void launch_orth_range(hipStream_t st, int dim, const OrthView& t, const uint32_t* boxes, uint64_t nb,
                       const uint32_t* order, uint64_t* counts, const uint64_t* offsets, uint32_t* ids) {
    if (nb == 0) return;
    const dim3 g(blocks_for(nb, 256));
    const bool rep = ids != nullptr;
    if (dim == 2) {
        if (rep) hipLaunchKernelGGL((k_orth_range<2, true>), g, dim3(256), 0, st, t, boxes, nb, order, counts, offsets, ids);
        else hipLaunchKernelGGL((k_orth_range<2, false>), g, dim3(256), 0, st, t, boxes, nb, order, counts, offsets, ids);
    } else {
        if (rep) hipLaunchKernelGGL((k_orth_range<3, true>), g, dim3(256), 0, st, t, boxes, nb, order, counts, offsets, ids);
        else hipLaunchKernelGGL((k_orth_range<3, false>), g, dim3(256), 0, st, t, boxes, nb, order, counts, offsets, ids);
    }
}

}  // namespace psi
