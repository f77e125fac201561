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

// ------------------------------------------------------------ packed boxes
__device__ __forceinline__ bool box_leaf(uint4 v) { return (v.y >> 31) != 0; }

template <int D> __device__ __forceinline__ void box_unpack(uint4 v, uint32_t* lo, uint32_t* hi) {
    const uint64_t a = ((uint64_t)v.y << 32) | v.x, b = ((uint64_t)v.w << 32) | v.z;
    constexpr int W = BoxBits<D>::W;
    constexpr uint64_t M = (1ull << W) - 1;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = (uint32_t)((a >> (d * W)) & M);
        hi[d] = (uint32_t)((b >> (d * W)) & M);
    }
}

template <int D> __device__ __forceinline__ uint4 box_pack(const uint32_t* lo, const uint32_t* hi, bool leaf) {
    constexpr int W = BoxBits<D>::W;
    uint64_t a = leaf ? 1ull << 63 : 0ull, b = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        a |= (uint64_t)lo[d] << (d * W);
        b |= (uint64_t)hi[d] << (d * W);
    }
    return make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
}

template <int D> __device__ __forceinline__ uint64_t box_dist2(const uint32_t* q, uint4 v) {
    uint32_t lo[D], hi[D];
    box_unpack<D>(v, lo, hi);
    uint64_t s = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const uint32_t x = q[d] < lo[d] ? lo[d] - q[d] : (q[d] > hi[d] ? q[d] - hi[d] : 0u);
        s += (uint64_t)x * x;
    }
    return s;
}

// --------------------------------------------------------------- leaf cut
constexpr uint32_t OM_HALO = 32;  // keys loaded beyond each side of a tile (leaf size <= 32)
constexpr uint32_t OM_PER = ORTH_TILE / 256;
static_assert(OM_PER == 8, "a thread's marks are stored as one 8-byte word");

template <int D>
__global__ __launch_bounds__(256) void k_orth_mark(const uint64_t* __restrict__ sk, const uint32_t* __restrict__ sid,
                                                   uint64_t n, uint32_t phi, uint8_t* __restrict__ mark,
                                                   uint32_t* __restrict__ tile_cnt, uint4* __restrict__ pts,
                                                   uint32_t* __restrict__ ids) {
    __shared__ uint64_t s_k[ORTH_TILE + 2 * OM_HALO];  // key at position base - OM_HALO + x
    __shared__ uint8_t s_cp[ORTH_TILE + OM_HALO];      // 1 + levels shared by keys j and j + phi
    __shared__ uint32_t s_w[4];
    const uint64_t base = (uint64_t)blockIdx.x * ORTH_TILE;
    {
        constexpr uint32_t SPAN = ORTH_TILE + 2 * OM_HALO, NLD = (SPAN + 255) / 256;
        uint64_t kk[NLD];  // all of a thread's loads in flight at once
#pragma unroll
        for (uint32_t r = 0; r < NLD; ++r) {
            const uint32_t x = threadIdx.x + 256 * r;
            const int64_t g = (int64_t)base - (int64_t)OM_HALO + x;
            kk[r] = (x < SPAN && g >= 0 && (uint64_t)g < n) ? sk[g] : 0ull;
        }
#pragma unroll
        for (uint32_t r = 0; r < NLD; ++r) {
            const uint32_t x = threadIdx.x + 256 * r;
            if (x < SPAN) s_k[x] = kk[r];
        }
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
    // positions y0 + u of the tile; position y's windows j in [y - phi, y]
    // are s_cp[y + OM_HALO - phi .. y + OM_HALO]. For phi >= 7 the eight
    // windows share [y0 + 39 - phi, y0 + 32]; the rest is a suffix maximum on
    // the left and a prefix maximum on the right.
    const uint32_t y0 = threadIdx.x * OM_PER;
    uint32_t m1[OM_PER];
    if (phi >= 7) {
        uint32_t core = 0;
        for (uint32_t x = y0 + 39 - phi; x <= y0 + 32; ++x) core = max(core, (uint32_t)s_cp[x]);
        uint32_t lf = 0, rg = 0;
        m1[OM_PER - 1] = core;
#pragma unroll
        for (int u = OM_PER - 2; u >= 0; --u) {
            lf = max(lf, (uint32_t)s_cp[y0 + u + 32 - phi]);
            m1[u] = max(core, lf);
        }
#pragma unroll
        for (uint32_t u = 1; u < OM_PER; ++u) {
            rg = max(rg, (uint32_t)s_cp[y0 + u + 32]);
            m1[u] = max(m1[u], rg);
        }
    } else {
#pragma unroll
        for (uint32_t u = 0; u < OM_PER; ++u) {
            uint32_t m = 0;
            for (uint32_t x = y0 + u + OM_HALO - phi; x <= y0 + u + OM_HALO; ++x) m = max(m, (uint32_t)s_cp[x]);
            m1[u] = m;
        }
    }
    uint64_t word = 0;
    uint32_t c = 0;
#pragma unroll
    for (uint32_t u = 0; u < OM_PER; ++u) {
        const uint64_t i = base + y0 + u;
        if (i < n) {
            const uint32_t l = min(m1[u], OrthBits<D>::W);
            const bool st = i == 0 || common_levels<D>(s_k[y0 + u + OM_HALO - 1], s_k[y0 + u + OM_HALO]) < l;
            word |= (uint64_t)(l | (st ? 0x80u : 0u)) << (8 * u);
            c += st ? 1u : 0u;
        }
    }
    *reinterpret_cast<uint2*>(mark + base + y0) = make_uint2((uint32_t)word, (uint32_t)(word >> 32));
    const uint32_t incl = block_incl_scan256(c, s_w);
    if (threadIdx.x == 255) tile_cnt[blockIdx.x] = incl;
    // the points in key order, coordinates decoded from the keys
    uint32_t idv[OM_PER];
#pragma unroll
    for (uint32_t r = 0; r < OM_PER; ++r) {
        const uint64_t i = base + threadIdx.x + 256 * r;
        idv[r] = i < n ? sid[i] : 0u;
    }
#pragma unroll
    for (uint32_t r = 0; r < OM_PER; ++r) {
        const uint32_t y = threadIdx.x + 256 * r;
        const uint64_t i = base + y;
        if (i < n) {
            uint32_t p[3] = {0u, 0u, 0u};
            morton_point<D>(s_k[y + OM_HALO], p);
            pts[i] = make_uint4(p[0], p[1], D == 3 ? p[2] : 0u, idv[r]);
            ids[i] = idv[r];
        }
    }
}

// Second pass over a tile: the leaves' first positions, levels and keys,
// then their boxes. The tile's points, with OM_HALO positions beyond it, are
// decoded from the keys into LDS (three words per position: no bank
// conflicts); a thread per leaf reduces its run of points there. Only the
// tile's last leaf can end past the tile; if it is a leaf of equal points
// running past the staged positions, its thread reads on from global memory.
template <int D>
__global__ __launch_bounds__(256) void k_orth_leaves(const uint64_t* __restrict__ sk, uint64_t n,
                                                     const uint8_t* __restrict__ mark,
                                                     const uint32_t* __restrict__ tile_off,
                                                     uint32_t* __restrict__ lstart, uint8_t* __restrict__ llev,
                                                     uint64_t* __restrict__ fkey, uint4* __restrict__ lbox) {
    constexpr uint32_t SPAN = ORTH_TILE + OM_HALO;
    __shared__ uint32_t s_p[SPAN * 3];
    __shared__ uint16_t s_st[ORTH_TILE];  // tile position of the tile's k-th leaf start
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_nl;
    const uint64_t base = (uint64_t)blockIdx.x * ORTH_TILE;
    constexpr uint32_t NLD = (SPAN + 255) / 256;
    uint64_t kk[NLD];  // all of a thread's loads in flight before any decode
#pragma unroll
    for (uint32_t r = 0; r < NLD; ++r) {
        const uint32_t x = threadIdx.x + 256 * r;
        const uint64_t g = base + x;
        kk[r] = (x < SPAN && g < n) ? sk[g] : 0ull;
    }
#pragma unroll
    for (uint32_t r = 0; r < NLD; ++r) {
        const uint32_t x = threadIdx.x + 256 * r;
        if (x < SPAN) {
            uint32_t p[3] = {0u, 0u, 0u};
            morton_point<D>(kk[r], p);
            s_p[3 * x] = p[0];
            s_p[3 * x + 1] = p[1];
            s_p[3 * x + 2] = p[2];
        }
    }
    const uint32_t y0 = threadIdx.x * OM_PER;
    const uint2 mm = *reinterpret_cast<const uint2*>(mark + base + y0);
    const uint64_t word = ((uint64_t)mm.y << 32) | mm.x;
    const uint32_t c = (uint32_t)__popcll(word & 0x8080808080808080ull);
    const uint32_t incl = block_incl_scan256(c, s_w);
    if (threadIdx.x == 255) s_nl = incl;
    const uint32_t t0 = tile_off[blockIdx.x];
    uint32_t k = incl - c;
#pragma unroll
    for (uint32_t u = 0; u < OM_PER; ++u) {
        const uint32_t b = (uint32_t)(word >> (8 * u)) & 0xFFu;
        if (b & 0x80u) {
            const uint64_t i = base + y0 + u;
            lstart[t0 + k] = (uint32_t)i;
            llev[t0 + k] = (uint8_t)(b & 0x7Fu);
            fkey[t0 + k] = sk[i];
            s_st[k] = (uint16_t)(y0 + u);
            ++k;
        }
    }
    __syncthreads();
    const uint32_t nl = s_nl;
    const uint64_t tile_end = min<uint64_t>(ORTH_TILE, n - base);
    for (uint32_t j = threadIdx.x; j < nl; j += 256) {
        const uint32_t y = s_st[j];
        uint32_t lo[D], hi[D];
#pragma unroll
        for (int d = 0; d < D; ++d) lo[d] = hi[d] = s_p[3 * y + d];
        if (j + 1 < nl) {
            const uint32_t ye = s_st[j + 1];
            for (uint32_t x = y + 1; x < ye; ++x) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    lo[d] = min(lo[d], s_p[3 * x + d]);
                    hi[d] = max(hi[d], s_p[3 * x + d]);
                }
            }
        } else {  // the tile's last leaf: up to the next start, which may lie past the tile
            uint64_t g = base + y + 1;
            for (; g < n && (g < base + tile_end || !(mark[g] & 0x80u)); ++g) {
                const uint64_t x = g - base;
                uint32_t p[3];
                if (x < SPAN) {
                    p[0] = s_p[3 * x];
                    p[1] = s_p[3 * x + 1];
                    p[2] = s_p[3 * x + 2];
                } else {
                    morton_point<D>(sk[g], p);
                }
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    lo[d] = min(lo[d], p[d]);
                    hi[d] = max(hi[d], p[d]);
                }
            }
        }
        lbox[t0 + j] = box_pack<D>(lo, hi, true);
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
    if (threadIdx.x == 0) {  // one atomic only where the block raises the maximum seen so far
        const uint32_t m = max(max(s_m[0], s_m[1]), max(s_m[2], s_m[3]));
        if (m > __hip_atomic_load(maxlev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(maxlev, m);
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_orth_nodes(const uint8_t* __restrict__ llev, const uint64_t* __restrict__ fkey,
                                                    const uint32_t* __restrict__ lstart,
                                                    const uint32_t* __restrict__ base, uint32_t L, uint32_t n,
                                                    uint64_t N, const uint4* __restrict__ lbox,
                                                    uint4* __restrict__ box, uint2* __restrict__ link,
                                                    uint32_t* __restrict__ first, uint8_t* __restrict__ lev) {
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
        // first later leaf outside the cell: doubling steps, then bisection
        uint32_t in = t, out = L;
        for (uint32_t step = 1;; step <<= 1) {
            const uint64_t pr = (uint64_t)t + step;
            if (pr >= L) break;
            if ((fkey[pr] >> sh) != cell) {
                out = (uint32_t)pr;
                break;
            }
            in = (uint32_t)pr;
        }
        while (out - in > 1) {
            const uint32_t mid = in + ((out - in) >> 1);
            if ((fkey[mid] >> sh) == cell) in = mid;
            else out = mid;
        }
        const uint64_t v = b + (l - s);
        link[v] = make_uint2(out < L ? base[out] : (uint32_t)N, (out < L ? lstart[out] : n) - pb);
        box[v] = make_uint4(0u, 0u, 0u, 0u);
        first[v] = pb;
        lev[v] = (uint8_t)l;
    }
    const uint64_t v = b + (s <= lv ? lv - s : 0u);
    box[v] = lbox[t];
    link[v] = make_uint2(pb, pe - pb);
    first[v] = pb;
    lev[v] = 0xFF;
}

template <int D>
__global__ __launch_bounds__(256) void k_orth_boxes(uint32_t level, uint64_t N, const uint8_t* __restrict__ lev,
                                                    uint4* __restrict__ box, const uint2* __restrict__ link) {
    // sixteen nodes per thread: one 16-byte read of their levels
    const uint64_t v0 = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    if (v0 >= N) return;
    uint32_t match = 0;  // bit u: node v0 + u is an interior node of this level
    if (v0 + 16 <= N) {
        const uint4 w = *reinterpret_cast<const uint4*>(lev + v0);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int u = 0; u < 16; ++u) match |= (((ws[u >> 2] >> (8 * (u & 3))) & 0xFFu) == level ? 1u : 0u) << u;
    } else {
        for (int u = 0; v0 + u < N; ++u) match |= (lev[v0 + u] == level ? 1u : 0u) << u;
    }
    while (match) {
        const int u = __builtin_ctz(match);
        match &= match - 1;
        const uint64_t v = v0 + u;
        const uint64_t end = min<uint64_t>(link[v].x, N);
        uint32_t lo[D], hi[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = 0xFFFFFFFFu;
            hi[d] = 0u;
        }
        uint64_t c = v + 1;
        while (c < end) {  // the children: first child v + 1, then each one's end
            const uint4 bx = box[c];
            uint32_t a[D], z[D];
            box_unpack<D>(bx, a, z);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                lo[d] = min(lo[d], a[d]);
                hi[d] = max(hi[d], z[d]);
            }
            const uint64_t nx = box_leaf(bx) ? c + 1 : (uint64_t)link[c].x;
            c = nx > c ? nx : c + 1;
        }
        box[v] = box_pack<D>(lo, hi, false);
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_orth_export(const uint4* __restrict__ box, const uint2* __restrict__ link,
                                                     uint64_t N, uint32_t* __restrict__ out) {
    const uint64_t v = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= N) return;
    const uint4 bx = box[v];
    uint32_t lo[D], hi[D];
    box_unpack<D>(bx, lo, hi);
    const uint2 lk = link[v];
    uint32_t* o = out + v * 8;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        o[d] = d < D ? lo[d] : 0u;
        o[3 + d] = d < D ? hi[d] : 0u;
    }
    o[6] = lk.x;
    o[7] = lk.y | (box_leaf(bx) ? 0x80000000u : 0u);
}

// ------------------------------------------------------------------ queries
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

constexpr uint32_t ORTH_SEED = 64;  // points scanned around the query's key before the walk

// Lane per query. The leaves around the query's own Morton position (the
// one holding it, then its neighbours in key order until they hold
// ORTH_SEED points: one contiguous run of the point array) are scanned first
// to start with a small k-th distance; the preorder walk then skips them.
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
        uint32_t ja = j, jb = j;
        uint32_t p0 = t.lstart[j], p1 = j + 1 < t.L ? t.lstart[j + 1] : t.n;
        while (p1 - p0 < ORTH_SEED && (ja > 0 || jb + 1 < t.L)) {
            if (ja > 0) p0 = t.lstart[--ja];
            if (jb + 1 < t.L) {
                ++jb;
                p1 = jb + 1 < t.L ? t.lstart[jb + 1] : t.n;
            }
        }
        orth_scan<D, K>(t.pts, p0, p1, q, bd, bi);
        uint64_t v = 0;
        while (v < t.N) {
            const uint4 bx = t.box[v];
            const bool leaf = box_leaf(bx);
            if (box_dist2<D>(q, bx) <= bd[K - 1]) {
                if (leaf) {
                    const uint2 lk = t.link[v];
                    if (lk.x < p0 || lk.x >= p1) orth_scan<D, K>(t.pts, lk.x, lk.x + lk.y, q, bd, bi);
                }
                ++v;
            } else {
                v = leaf ? v + 1 : max<uint64_t>(t.link[v].x, v + 1);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        out_ids[qi * K + j] = bi[j];
        out_d2[qi * K + j] = bd[j];
    }
}

// ----------------------------------------------------- kNN, wave per query
// For k > 16: the k best pairs of a query live in LDS, ascending, in two
// copies (the merge writes the other one). A batch of up to 64 points (one per
// lane) is merged in: the points that beat the current k-th pair are ranked
// among themselves, each list entry and each candidate finds its new place by
// binary search in the other sequence.
constexpr int OKW_WAVES = 4;

template <int KMAX>
struct OrthKList {
    uint64_t (*d)[KMAX];  // [2][KMAX]
    uint32_t (*i)[KMAX];
    uint64_t* cd;         // [64] candidates
    uint32_t* ci;
};

template <int D, int KMAX>
__device__ __forceinline__ void orth_merge64(const OrthKList<KMAX>& L, int& cur, uint32_t k, bool valid, uint4 P,
                                             const uint32_t* q) {
    const uint32_t lane = lane_id();
    uint64_t dd = PAD_D2;
    uint32_t id = PAD_ID;
    bool cand = false;
    if (valid) {
        const uint32_t p[3] = {P.x, P.y, P.z};
        dd = pt_dist<D>(q, p);
        id = P.w;
        cand = pair_less(dd, id, L.d[cur][k - 1], L.i[cur][k - 1]);
    }
    const uint64_t cm = ballot(cand);
    if (cm == 0) return;
    const uint32_t nc = (uint32_t)__popcll(cm);
    if (cand) {
        const uint32_t slot = count_below(cm);
        L.cd[slot] = dd;
        L.ci[slot] = id;
    }
    __builtin_amdgcn_wave_barrier();
    uint32_t cpos = 0, rank = 0;
    if (cand) {
        for (uint32_t x = 0; x < nc; ++x) rank += pair_less(L.cd[x], L.ci[x], dd, id) ? 1u : 0u;
        uint32_t lo = 0, hi = k;  // list entries below the candidate
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pair_less(L.d[cur][mid], L.i[cur][mid], dd, id)) lo = mid + 1;
            else hi = mid;
        }
        cpos = rank + lo;
    }
    __builtin_amdgcn_wave_barrier();  // every lane has read the unsorted candidates
    if (cand) {
        L.cd[rank] = dd;
        L.ci[rank] = id;
    }
    __builtin_amdgcn_wave_barrier();
    const int nxt = cur ^ 1;
    for (uint32_t x = lane; x < k; x += 64) {
        const uint64_t ld = L.d[cur][x];
        const uint32_t li = L.i[cur][x];
        uint32_t lo = 0, hi = nc;  // candidates below list entry x
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pair_less(L.cd[mid], L.ci[mid], ld, li)) lo = mid + 1;
            else hi = mid;
        }
        if (x + lo < k) {
            L.d[nxt][x + lo] = ld;
            L.i[nxt][x + lo] = li;
        }
    }
    if (cand && cpos < k) {
        L.d[nxt][cpos] = dd;
        L.i[nxt][cpos] = id;
    }
    __builtin_amdgcn_wave_barrier();
    cur = nxt;
}

// The walk takes 64 preorder nodes per step, as the range kernel does: a
// node is skipped when an earlier pruned interior node's subtree covers it;
// the leaves left within the k-th distance are scanned in order, 64 points
// at a time, each rechecked against the k-th distance of the moment.
template <int D, int KMAX>
__global__ __launch_bounds__(256) void k_orth_knn_wave(OrthView t, const uint32_t* __restrict__ qp,
                                                       const uint64_t* __restrict__ qkeys, uint64_t nq,
                                                       const uint32_t* __restrict__ order, uint32_t k,
                                                       uint32_t* __restrict__ out_ids,
                                                       uint64_t* __restrict__ out_d2) {
    __shared__ uint64_t s_d[OKW_WAVES][2][KMAX];
    __shared__ uint32_t s_i[OKW_WAVES][2][KMAX];
    __shared__ uint64_t s_cd[OKW_WAVES][64];
    __shared__ uint32_t s_ci[OKW_WAVES][64];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = lane_id();
    const uint64_t tq = (uint64_t)blockIdx.x * OKW_WAVES + w;
    if (tq >= nq) return;
    const uint64_t qi = order ? order[tq] : tq;
    uint32_t q[D];
#pragma unroll
    for (int d = 0; d < D; ++d) q[d] = qp[qi * D + d];
    for (uint32_t x = lane; x < KMAX; x += 64) {
        s_d[w][0][x] = PAD_D2;
        s_i[w][0][x] = PAD_ID;
    }
    __builtin_amdgcn_wave_barrier();
    const OrthKList<KMAX> Lst{s_d[w], s_i[w], s_cd[w], s_ci[w]};
    int cur = 0;
    if (t.N > 0 && t.L > 0) {
        const uint64_t key = qkeys[qi];
        uint32_t lo = 0, hi = t.L;
        while (lo < hi) {
            const uint32_t mid = lo + ((hi - lo) >> 1);
            if (t.fkey[mid] <= key) lo = mid + 1;
            else hi = mid;
        }
        const uint32_t j = lo ? lo - 1 : 0u;
        const uint32_t want = max(ORTH_SEED, 2 * k);
        uint32_t ja = j, jb = j;
        uint32_t p0 = t.lstart[j], p1 = j + 1 < t.L ? t.lstart[j + 1] : t.n;
        while (p1 - p0 < want && (ja > 0 || jb + 1 < t.L)) {
            if (ja > 0) p0 = t.lstart[--ja];
            if (jb + 1 < t.L) {
                ++jb;
                p1 = jb + 1 < t.L ? t.lstart[jb + 1] : t.n;
            }
        }
        for (uint32_t e0 = p0; e0 < p1; e0 += 64) {
            const uint32_t e = e0 + lane;
            const bool ok = e < p1;
            orth_merge64<D, KMAX>(Lst, cur, k, ok, ok ? t.pts[e] : make_uint4(0u, 0u, 0u, 0u), q);
        }
        uint64_t v = 0;
        while (v < t.N) {
            const uint64_t kth = s_d[w][cur][k - 1];
            const uint64_t i = v + lane;
            const bool valid = i < t.N;
            const uint4 bx = valid ? t.box[i] : make_uint4(0u, 0u, 0u, 0u);
            const bool leaf = box_leaf(bx);
            const uint64_t bd = valid ? box_dist2<D>(q, bx) : PAD_D2;
            const bool pruned = valid && bd > kth;
            const uint32_t jend = (pruned && !leaf) ? t.link[i].x : 0u;
            uint32_t incl = jend;  // inclusive prefix maximum of pruned subtree ends
#pragma unroll
            for (int sft = 1; sft < 64; sft <<= 1) {
                const uint32_t y = shfl_u32(incl, (int)lane - sft);
                if (lane >= (uint32_t)sft) incl = max(incl, y);
            }
            uint32_t excl = shfl_u32(incl, (int)lane - 1);
            if (lane == 0) excl = 0;
            const bool on = valid && (uint64_t)excl <= i;
            const uint32_t far = __builtin_amdgcn_readlane((int)incl, 63);
            uint64_t m = ballot(on && leaf && !pruned);
            while (m) {
                const uint32_t x = (uint32_t)__builtin_ctzll(m);
                m &= m - 1;
                const uint64_t dx = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(bd >> 32), (int)x) << 32) |
                                    (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)bd, (int)x);
                if (dx > s_d[w][cur][k - 1]) continue;
                const uint2 lk = t.link[v + x];
                if (lk.x >= p0 && lk.x < p1) continue;  // a seed leaf
                for (uint32_t e0 = lk.x; e0 < lk.x + lk.y; e0 += 64) {
                    const uint32_t e = e0 + lane;
                    const bool ok = e < lk.x + lk.y;
                    orth_merge64<D, KMAX>(Lst, cur, k, ok, ok ? t.pts[e] : make_uint4(0u, 0u, 0u, 0u), q);
                }
            }
            v = max<uint64_t>(v + 64, (uint64_t)far);
        }
    }
    for (uint32_t x = lane; x < k; x += 64) {
        out_ids[qi * k + x] = s_i[w][cur][x];
        out_d2[qi * k + x] = s_d[w][cur][x];
    }
}

// Wave per box. The wave takes the preorder nodes 64 at a time from the
// current position v (one node per lane, coalesced). A node is on the walk
// unless an earlier node of the window is an interior node whose subtree is
// decided by its box alone (apart from the query box, or inside it) and whose
// subtree reaches past it: subtrees nest, so an exclusive prefix maximum of
// those subtree ends over the lanes tells every lane whether it is skipped.
// The next window starts at v + 64 or past the farthest such subtree. On the
// walk: nodes inside the box add their counts (reports copy their ids, whole
// subtrees being contiguous in the point array, one node at a time by the
// whole wave); the points of the window's leaves that straddle the box are
// scanned one per lane, concatenated across leaves. The walk starts at the deepest node whose cell holds the whole
// box (the cell of the levels the Morton keys of the two corners share): every
// point in the box is below it.
constexpr int ORW_WAVES = 4;

// Preorder range [v0, v1) of the node whose cell is the level-ls cell holding
// key kl, or an empty range if that cell holds no point. A leaf whose cell
// contains it stands for it.
template <int D>
__device__ __forceinline__ void orth_cell_node(const OrthView& t, uint64_t kl, uint32_t ls, uint64_t& v0,
                                               uint64_t& v1) {
    v0 = v1 = 0;
    const uint32_t sh = OrthBits<D>::KB - ls * D;
    const uint64_t cell = kl >> sh, cstart = cell << sh;
    uint32_t lo = 0, hi = t.L;  // first leaf whose first key is >= the cell's start
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (t.fkey[mid] < cstart) lo = mid + 1;
        else hi = mid;
    }
    const uint32_t t1 = lo;
    if (t1 > 0) {  // the leaf before it may hold the whole cell
        const uint32_t tp = t1 - 1, lvp = t.llev[tp], shp = OrthBits<D>::KB - lvp * D;
        if (lvp <= ls && (t.fkey[tp] >> shp) == (cstart >> shp)) {
            const uint32_t s = open_from<D>(t.fkey, tp);
            v0 = (uint64_t)t.base[tp] + (s <= lvp ? lvp - s : 0u);
            v1 = v0 + 1;
            return;
        }
    }
    if (t1 < t.L && (t.fkey[t1] >> sh) == cell) {
        const uint32_t lv = t.llev[t1], s = open_from<D>(t.fkey, t1);
        if (lv <= ls) {  // leaf t1 holds the cell
            v0 = (uint64_t)t.base[t1] + (s <= lv ? lv - s : 0u);
            v1 = v0 + 1;
        } else if (s <= ls) {  // the interior node of level ls opened at t1
            v0 = (uint64_t)t.base[t1] + (ls - s);
            v1 = t.link[v0].x;
        } else {  // not reached for a consistent tree: walk everything
            v0 = 0;
            v1 = t.N;
        }
    }
}

template <int D, bool REPORT>
__global__ __launch_bounds__(256) void k_orth_range(OrthView t, const uint32_t* __restrict__ boxes, uint64_t nb,
                                                    const uint32_t* __restrict__ order, uint64_t* __restrict__ counts,
                                                    const uint64_t* __restrict__ offsets, uint32_t* __restrict__ out) {
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = lane_id();
    const uint64_t bx = (uint64_t)blockIdx.x * ORW_WAVES + w;
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
    uint64_t cnt_lane = 0, cnt = 0, o = 0, lim = 0;
    if (REPORT) {
        o = offsets[b];
        lim = offsets[b + 1];
    }
    // corners clamped to the coordinate domain (no point lies outside it)
    uint32_t clo[3] = {0u, 0u, 0u}, chi[3] = {0u, 0u, 0u};
#pragma unroll
    for (int d = 0; d < D; ++d) {
        constexpr uint32_t top = (1u << OrthBits<D>::W) - 1u;
        empty = empty || lo[d] > top;
        clo[d] = lo[d];
        chi[d] = min(hi[d], top);
    }
    uint64_t v = 0, vend = 0;
    if (!empty && t.N > 0) {
        const uint64_t kl = morton_key<D>(clo), kh = morton_key<D>(chi);
        orth_cell_node<D>(t, kl, common_levels<D>(kl, kh), v, vend);
    }
    while (v < vend) {
        const uint64_t i = v + lane;
        const bool valid = i < vend;
        uint4 nb4 = make_uint4(0u, 0u, 0u, 0u);
        uint2 lk = make_uint2(0u, 0u);
        if (valid) {
            nb4 = t.box[i];
            lk = t.link[i];
        }
        const bool leaf = box_leaf(nb4);
        uint32_t rl[D], rh[D];
        box_unpack<D>(nb4, rl, rh);
        bool inside = valid, apart = !valid;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            apart = apart || rh[d] < lo[d] || rl[d] > hi[d];
            inside = inside && lo[d] <= rl[d] && rh[d] <= hi[d];
        }
        const uint32_t jend = (valid && !leaf && (apart || inside)) ? lk.x : 0u;
        uint32_t incl = jend;  // inclusive prefix maximum over the lanes
#pragma unroll
        for (int s = 1; s < 64; s <<= 1) {
            const uint32_t y = shfl_u32(incl, (int)lane - s);
            if (lane >= (uint32_t)s) incl = max(incl, y);
        }
        uint32_t excl = shfl_u32(incl, (int)lane - 1);
        if (lane == 0) excl = 0;
        const bool on = valid && (uint64_t)excl <= i;
        const uint32_t far = __builtin_amdgcn_readlane((int)incl, 63);
        // whole subtrees inside the box
        const bool take = on && inside && !apart;
        if (!REPORT) {
            cnt_lane += take ? lk.y : 0u;
        } else {
            uint64_t m = ballot(take);
            while (m) {
                const uint32_t x = (uint32_t)__builtin_ctzll(m);
                m &= m - 1;
                const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)lk.y, (int)x);
                const uint32_t pb = t.first[v + x];
                for (uint32_t e = lane; e < c; e += 64) {
                    const uint64_t dst = o + e;
                    if (dst < lim) out[dst] = t.ids[pb + e];
                }
                o += c;
            }
        }
        // leaves straddling the box: their points, concatenated in lane
        // order, one point per lane per step
        const bool strad = on && leaf && !inside && !apart;
        const uint32_t lc = strad ? lk.y : 0u;
        uint32_t run = lc;  // inclusive scan of the counts over the lanes
#pragma unroll
        for (int sft = 1; sft < 64; sft <<= 1) {
            const uint32_t y = shfl_u32(run, (int)lane - sft);
            if (lane >= (uint32_t)sft) run += y;
        }
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)run, 63);
        for (uint32_t e0 = 0; e0 < tot; e0 += 64) {
            const uint32_t e = e0 + lane;
            uint32_t a = 0, z = 63;  // the first lane whose run end passes e
#pragma unroll
            for (int it = 0; it < 6; ++it) {
                const uint32_t mid = (a + z) >> 1;
                const uint32_t ev = shfl_u32(run, (int)mid);
                if (a < z) {
                    if (ev > e) z = mid;
                    else a = mid + 1;
                }
            }
            const uint32_t src = shfl_u32(lk.x, (int)a), p0 = shfl_u32(run - lc, (int)a);
            bool in = false;
            uint32_t id = 0;
            if (e < tot) {
                const uint4 P = t.pts[src + (e - p0)];
                const uint32_t p[3] = {P.x, P.y, P.z};
                in = true;
#pragma unroll
                for (int d = 0; d < D; ++d) in = in && lo[d] <= p[d] && p[d] <= hi[d];
                id = P.w;
            }
            const uint64_t hit = ballot(in);
            if (REPORT && in) {
                const uint64_t dst = o + count_below(hit);
                if (dst < lim) out[dst] = id;
            }
            if (REPORT) o += (uint32_t)__popcll(hit);
            else cnt += (uint32_t)__popcll(hit);
        }
        v = max<uint64_t>(v + 64, (uint64_t)far);
    }
    if (!REPORT) {
        for (int s = 32; s >= 1; s >>= 1) cnt_lane += shfl_u64(cnt_lane, (int)(lane ^ (uint32_t)s));
        if (lane == 0) counts[b] = cnt + cnt_lane;
    }
}

// ------------------------------------------------------------------ updates
// The tree is canonical (its shape depends only on the point set), so a batch
// update produces the new set's sorted (key, id) pairs by a merge or a
// compaction of the old order, and the tree is cut again from them.

// Place of each new pair among the old points: the number of old keys <= its
// key (every old id is smaller than every new one, so an old point with an
// equal key comes first); hist[place] counts them.
template <int D>
__global__ __launch_bounds__(256) void k_orth_place(const uint4* __restrict__ pts, uint64_t n,
                                                    const uint64_t* __restrict__ bk, uint64_t m,
                                                    uint32_t* __restrict__ place, uint32_t* __restrict__ hist) {
    const uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const uint64_t key = bk[j];
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        const uint4 P = pts[mid];
        const uint32_t p[3] = {P.x, P.y, P.z};
        if (morton_key<D>(p) <= key) lo = mid + 1;
        else hi = mid;
    }
    place[j] = (uint32_t)lo;
    atomicAdd(&hist[lo], 1u);
}

// Merged order: old point i moves up by the new pairs placed at or before it
// (hscan[i] + hist[i]), new pair j lands after place[j] old points and j new
// ones.
template <int D>
__global__ __launch_bounds__(256) void k_orth_merge(const uint4* __restrict__ pts, uint64_t n,
                                                    const uint32_t* __restrict__ hist,
                                                    const uint32_t* __restrict__ hscan,
                                                    const uint64_t* __restrict__ bk, const uint32_t* __restrict__ bid,
                                                    const uint32_t* __restrict__ place, uint64_t m,
                                                    uint64_t* __restrict__ mk, uint32_t* __restrict__ mi) {
    const uint64_t x = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (x < n) {
        const uint64_t dst = x + hscan[x] + hist[x];
        const uint4 P = pts[x];
        const uint32_t p[3] = {P.x, P.y, P.z};
        mk[dst] = morton_key<D>(p);
        mi[dst] = P.w;
    } else if (x < n + m) {
        const uint64_t j = x - n, dst = place[j] + j;
        mk[dst] = bk[j];
        mi[dst] = bid[j];
    }
}

// Clears the live bits of the batch's ids and counts the bits that were set.
// The entry that cleared a bit finds its point in the key order (binary
// search for (key, id), the key from the id's key table) and clears that
// position's keep flag.
template <int D>
__global__ __launch_bounds__(256) void k_orth_kill(const uint32_t* __restrict__ dids, uint64_t m, uint32_t next_id,
                                                   uint32_t* __restrict__ alive, const uint64_t* __restrict__ idkey,
                                                   const uint4* __restrict__ pts, uint64_t n,
                                                   uint32_t* __restrict__ keep, unsigned long long* __restrict__ removed,
                                                   uint32_t* __restrict__ err) {
    const uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    bool hit = false;
    if (j < m) {
        const uint32_t id = dids[j];
        if (id < next_id) {
            const uint32_t bit = 1u << (id & 31u);
            hit = (atomicAnd(&alive[id >> 5], ~bit) & bit) != 0;
            if (hit) {
                const uint64_t key = idkey[id];
                uint64_t lo = 0, hi = n;
                while (lo < hi) {
                    const uint64_t mid = lo + ((hi - lo) >> 1);
                    const uint4 P = pts[mid];
                    const uint32_t p[3] = {P.x, P.y, P.z};
                    if (pair_less(morton_key<D>(p), P.w, key, id)) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < n && pts[lo].w == id) keep[lo] = 0u;
                else atomicOr(err, ERR_ORTH);
            }
        }
    }
    const uint64_t b = ballot(hit);
    if (lane_id() == 0 && b) atomicAdd(removed, (unsigned long long)__popcll(b));
}

template <int D>
__global__ __launch_bounds__(256) void k_orth_compact(const uint4* __restrict__ pts, uint64_t n,
                                                      const uint32_t* __restrict__ flag,
                                                      const uint32_t* __restrict__ pos, uint64_t* __restrict__ mk,
                                                      uint32_t* __restrict__ mi) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const uint4 P = pts[i];
    const uint32_t p[3] = {P.x, P.y, P.z};
    mk[pos[i]] = morton_key<D>(p);
    mi[pos[i]] = P.w;
}

// Sets the live bits of ids [lo, hi): one thread per bitmap word; a word that
// starts at or after lo is written whole (its bits at or above hi cleared),
// the word holding older ids below lo is or-ed.
__global__ __launch_bounds__(256) void k_orth_alive(uint32_t* __restrict__ alive, uint32_t lo, uint32_t hi) {
    const uint64_t w = (uint64_t)(lo >> 5) + (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const uint64_t ws = w * 32;
    if (ws >= hi) return;
    const uint64_t a = ws > lo ? ws : lo, b = ws + 32 < hi ? ws + 32 : hi;
    const uint32_t nb = (uint32_t)(b - a);
    const uint32_t mask = (nb >= 32 ? 0xFFFFFFFFu : ((1u << nb) - 1u)) << (uint32_t)(a - ws);
    if (ws >= lo) alive[w] = mask;
    else alive[w] |= mask;
}

__global__ void k_orth_put64(unsigned long long* p, unsigned long long v) {
    if (threadIdx.x == 0) *p = v;
}

}  // namespace

void launch_orth_mark(hipStream_t st, int dim, const uint64_t* sk, const uint32_t* sid, uint64_t n, uint32_t phi,
                      uint8_t* mark, uint32_t* tile_cnt, uint4* pts, uint32_t* ids) {
    if (n == 0) return;
    const dim3 g(blocks_for(n, ORTH_TILE));
    if (dim == 2) hipLaunchKernelGGL((k_orth_mark<2>), g, dim3(256), 0, st, sk, sid, n, phi, mark, tile_cnt, pts, ids);
    else hipLaunchKernelGGL((k_orth_mark<3>), g, dim3(256), 0, st, sk, sid, n, phi, mark, tile_cnt, pts, ids);
}

void launch_orth_leaves(hipStream_t st, int dim, const uint64_t* sk, uint64_t n, const uint8_t* mark,
                        const uint32_t* tile_off, uint32_t* lstart, uint8_t* llev, uint64_t* fkey, uint4* lbox) {
    if (n == 0) return;
    const dim3 g(blocks_for(n, ORTH_TILE));
    if (dim == 2) hipLaunchKernelGGL((k_orth_leaves<2>), g, dim3(256), 0, st, sk, n, mark, tile_off, lstart, llev, fkey, lbox);
    else hipLaunchKernelGGL((k_orth_leaves<3>), g, dim3(256), 0, st, sk, n, mark, tile_off, lstart, llev, fkey, lbox);
}

void launch_orth_counts(hipStream_t st, int dim, const uint8_t* llev, const uint64_t* fkey, uint32_t L,
                        uint32_t* cnt1, uint32_t* maxlev, uint32_t* err) {
    if (L == 0) return;
    const dim3 g(blocks_for(L, 256));
    if (dim == 2) hipLaunchKernelGGL((k_orth_counts<2>), g, dim3(256), 0, st, llev, fkey, L, cnt1, maxlev, err);
    else hipLaunchKernelGGL((k_orth_counts<3>), g, dim3(256), 0, st, llev, fkey, L, cnt1, maxlev, err);
}

void launch_orth_nodes(hipStream_t st, int dim, const uint8_t* llev, const uint64_t* fkey, const uint32_t* lstart,
                       const uint32_t* base, uint32_t L, uint32_t n, uint64_t N, const uint4* lbox, uint4* box,
                       uint2* link, uint32_t* first, uint8_t* lev) {
    if (L == 0) return;
    const dim3 g(blocks_for(L, 256));
    if (dim == 2) hipLaunchKernelGGL((k_orth_nodes<2>), g, dim3(256), 0, st, llev, fkey, lstart, base, L, n, N, lbox, box, link, first, lev);
    else hipLaunchKernelGGL((k_orth_nodes<3>), g, dim3(256), 0, st, llev, fkey, lstart, base, L, n, N, lbox, box, link, first, lev);
}

void launch_orth_boxes(hipStream_t st, int dim, uint32_t level, uint64_t N, const uint8_t* lev, uint4* box,
                       const uint2* link) {
    if (N == 0) return;
    const dim3 g(blocks_for((N + 15) / 16, 256));
    if (dim == 2) hipLaunchKernelGGL((k_orth_boxes<2>), g, dim3(256), 0, st, level, N, lev, box, link);
    else hipLaunchKernelGGL((k_orth_boxes<3>), g, dim3(256), 0, st, level, N, lev, box, link);
}

void launch_orth_export(hipStream_t st, int dim, const uint4* box, const uint2* link, uint64_t N, uint32_t* out) {
    if (N == 0) return;
    const dim3 g(blocks_for(N, 256));
    if (dim == 2) hipLaunchKernelGGL((k_orth_export<2>), g, dim3(256), 0, st, box, link, N, out);
    else hipLaunchKernelGGL((k_orth_export<3>), g, dim3(256), 0, st, box, link, N, out);
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
        case 16: PSI_OK_(D, 16); break;                                                                  \
        default: {                                                                                       \
            const dim3 gw(blocks_for(nq, OKW_WAVES));                                                    \
            if (k <= 32) hipLaunchKernelGGL((k_orth_knn_wave<D, 32>), gw, dim3(256), 0, st, t, q, qkeys, nq, order, k, ids, d2); \
            else if (k <= 64) hipLaunchKernelGGL((k_orth_knn_wave<D, 64>), gw, dim3(256), 0, st, t, q, qkeys, nq, order, k, ids, d2); \
            else hipLaunchKernelGGL((k_orth_knn_wave<D, 128>), gw, dim3(256), 0, st, t, q, qkeys, nq, order, k, ids, d2); \
        }                                                                                                \
    }
    if (dim == 2) { PSI_OK_ALL(2) } else { PSI_OK_ALL(3) }
#undef PSI_OK_ALL
#undef PSI_OK_
}

void launch_orth_range(hipStream_t st, int dim, const OrthView& t, const uint32_t* boxes, uint64_t nb,
                       const uint32_t* order, uint64_t* counts, const uint64_t* offsets, uint32_t* ids) {
    if (nb == 0) return;
    const dim3 g(blocks_for(nb, ORW_WAVES));
    const bool rep = ids != nullptr;
    if (dim == 2) {
        if (rep) hipLaunchKernelGGL((k_orth_range<2, true>), g, dim3(256), 0, st, t, boxes, nb, order, counts, offsets, ids);
        else hipLaunchKernelGGL((k_orth_range<2, false>), g, dim3(256), 0, st, t, boxes, nb, order, counts, offsets, ids);
    } else {
        if (rep) hipLaunchKernelGGL((k_orth_range<3, true>), g, dim3(256), 0, st, t, boxes, nb, order, counts, offsets, ids);
        else hipLaunchKernelGGL((k_orth_range<3, false>), g, dim3(256), 0, st, t, boxes, nb, order, counts, offsets, ids);
    }
}

void launch_orth_place(hipStream_t st, int dim, const uint4* pts, uint64_t n, const uint64_t* bk, uint64_t m,
                       uint32_t* place, uint32_t* hist) {
    if (m == 0) return;
    const dim3 g(blocks_for(m, 256));
    if (dim == 2) hipLaunchKernelGGL((k_orth_place<2>), g, dim3(256), 0, st, pts, n, bk, m, place, hist);
    else hipLaunchKernelGGL((k_orth_place<3>), g, dim3(256), 0, st, pts, n, bk, m, place, hist);
}

void launch_orth_merge(hipStream_t st, int dim, const uint4* pts, uint64_t n, const uint32_t* hist,
                       const uint32_t* hscan, const uint64_t* bk, const uint32_t* bid, const uint32_t* place,
                       uint64_t m, uint64_t* mk, uint32_t* mi) {
    if (n + m == 0) return;
    const dim3 g(blocks_for(n + m, 256));
    if (dim == 2) hipLaunchKernelGGL((k_orth_merge<2>), g, dim3(256), 0, st, pts, n, hist, hscan, bk, bid, place, m, mk, mi);
    else hipLaunchKernelGGL((k_orth_merge<3>), g, dim3(256), 0, st, pts, n, hist, hscan, bk, bid, place, m, mk, mi);
}

void launch_orth_kill(hipStream_t st, int dim, const uint32_t* dids, uint64_t m, uint32_t next_id, uint32_t* alive,
                      const uint64_t* idkey, const uint4* pts, uint64_t n, uint32_t* keep,
                      unsigned long long* removed, uint32_t* err) {
    if (m == 0) return;
    const dim3 g(blocks_for(m, 256));
    if (dim == 2) hipLaunchKernelGGL((k_orth_kill<2>), g, dim3(256), 0, st, dids, m, next_id, alive, idkey, pts, n, keep, removed, err);
    else hipLaunchKernelGGL((k_orth_kill<3>), g, dim3(256), 0, st, dids, m, next_id, alive, idkey, pts, n, keep, removed, err);
}

void launch_orth_compact(hipStream_t st, int dim, const uint4* pts, uint64_t n, const uint32_t* flag,
                         const uint32_t* pos, uint64_t* mk, uint32_t* mi) {
    if (n == 0) return;
    const dim3 g(blocks_for(n, 256));
    if (dim == 2) hipLaunchKernelGGL((k_orth_compact<2>), g, dim3(256), 0, st, pts, n, flag, pos, mk, mi);
    else hipLaunchKernelGGL((k_orth_compact<3>), g, dim3(256), 0, st, pts, n, flag, pos, mk, mi);
}

void launch_orth_alive(hipStream_t st, uint32_t* alive, uint32_t lo, uint32_t hi) {
    if (hi <= lo) return;
    const uint64_t words = (((uint64_t)hi + 31) >> 5) - (lo >> 5);
    hipLaunchKernelGGL(k_orth_alive, dim3(blocks_for(words, 256)), dim3(256), 0, st, alive, lo, hi);
}

void launch_orth_put64(hipStream_t st, unsigned long long* p, unsigned long long v) {
    hipLaunchKernelGGL(k_orth_put64, dim3(1), dim3(64), 0, st, p, v);
}

}  // namespace psi
