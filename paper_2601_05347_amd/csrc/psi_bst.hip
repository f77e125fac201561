// The SPaC-tree in the paper's own shape (Alg. 3's BuildSorted): a binary
// search tree on (curve key, id) whose subtrees of at most phi points are
// wrapped into leaves and whose interior nodes each hold one point, the
// middle entry of their sorted range.
//
// The shape depends on n alone, so the GPU lays it out as an implicit heap
// (node v has children 2v + 1 and 2v + 2; children of a leaf are absent):
// node v's sorted range follows from the bits of v + 1 by the split rule
// (m = a + (b - a) / 2, left [a, m), right [m + 1, b)), one thread per node.
// A node's subtree holds exactly the entries of its range, in order, so a
// leaf is a run of the sorted arrays and a subtree inside a query box reports
// one contiguous run of ids. Boxes come bottom up, one launch per depth
// (a leaf's from its points; an interior node's from its children's and its
// pivot's).
//
// Batch updates (Alg. 4) keep the points sorted: an insert merges the
// batch's sorted pairs into the sorted arrays (each new entry's place by a
// binary search, each old entry's shift by a prefix sum), a delete compacts
// them; the shape is then laid out again for the new size. This gives the
// tree BuildSorted makes for the new set: perfectly balanced, where the
// paper's join-based updates keep it weight-balanced (the oracle runs those).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>

#include "../../include/psi.h"
#include "psi_index.h"
#include "psi_kern.h"

namespace psi {
namespace {

inline unsigned blocks_of(uint64_t n, unsigned per) {
    const uint64_t b = (n + per - 1) / per;
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(b, 1u << 20));
}

// Heap record: box and count as a NodeRec (cnt = entries in the subtree, 0
// for an absent node; slot = 1 for a leaf, 0 for an interior node), and the
// sorted range [a, b).
struct BstView {
    const NodeRec* node;
    const uint2* range;
    const uint32_t* pts;  // D words per entry, sorted order
    const uint32_t* ids;
    const uint64_t* keys;
    uint32_t n, depth;
};

// Range of heap node v (n entries, leaf wrap phi), or absent.
__device__ __forceinline__ bool bst_range(uint64_t v, uint32_t n, uint32_t phi, uint32_t& a, uint32_t& b) {
    const uint64_t x = v + 1;
    const int d = 63 - __builtin_clzll(x);  // depth
    a = 0;
    b = n;
    for (int s = d - 1; s >= 0; --s) {  // path from the root: bit s of x, 0 = left
        if (b - a <= phi) return false;  // an ancestor is a leaf
        const uint32_t m = a + (b - a) / 2;
        if ((x >> s) & 1u) a = m + 1;
        else b = m;
    }
    return true;
}

template <int D>
__global__ void k_bst_layout(uint32_t n, uint32_t phi, uint64_t H, NodeRec* __restrict__ node,
                             uint2* __restrict__ range, const uint32_t* __restrict__ pts) {
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < H; v += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t a, b;
        NodeRec r;
        for (int d = 0; d < 3; ++d) {
            r.lo[d] = 0xFFFFFFFFu;
            r.hi[d] = 0u;
        }
        r.cnt = 0;
        r.slot = 0;
        if (bst_range(v, n, phi, a, b) && b > a) {
            r.cnt = b - a;
            r.slot = b - a <= phi ? 1u : 0u;
            if (r.slot) {  // a leaf: its points' box
                for (uint32_t i = a; i < b; ++i)
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        const uint32_t c = pts[(uint64_t)i * D + d];
                        r.lo[d] = min(r.lo[d], c);
                        r.hi[d] = max(r.hi[d], c);
                    }
            }
            range[v] = make_uint2(a, b);
        } else {
            range[v] = make_uint2(0u, 0u);
        }
        if (D == 2 && r.cnt) r.lo[2] = 0u;
        node[v] = r;
    }
}

// Interior nodes of depth d: box = children's boxes and the pivot point.
template <int D>
__global__ void k_bst_inner(uint32_t d, NodeRec* __restrict__ node, const uint2* __restrict__ range,
                            const uint32_t* __restrict__ pts) {
    const uint64_t first = (1ull << d) - 1, cnt = 1ull << d;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t v = first + i;
        NodeRec r = node[v];
        if (r.cnt == 0 || r.slot == 1) continue;
        const uint2 ab = range[v];
        const uint32_t m = ab.x + (ab.y - ab.x) / 2;
        const NodeRec c0 = node[2 * v + 1], c1 = node[2 * v + 2];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const uint32_t p = pts[(uint64_t)m * D + k];
            r.lo[k] = min(p, min(c0.cnt ? c0.lo[k] : 0xFFFFFFFFu, c1.cnt ? c1.lo[k] : 0xFFFFFFFFu));
            r.hi[k] = max(p, max(c0.cnt ? c0.hi[k] : 0u, c1.cnt ? c1.hi[k] : 0u));
        }
        node[v] = r;
    }
}

// Points of the sorted entries: pts_out[i] = src[ids[i] - id_base].
template <int D>
__global__ void k_bst_gather(const uint32_t* __restrict__ ids, uint64_t n, const uint32_t* __restrict__ src,
                             uint32_t id_base, uint32_t* __restrict__ out) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t j = ids[i] - id_base;
#pragma unroll
        for (int d = 0; d < D; ++d) out[i * D + d] = src[j * D + d];
    }
}

__device__ __forceinline__ bool pair_lt(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

// Merge, step 1: each new entry's place among the old ones (first old entry
// above it) and a count of new entries per old position.
__global__ void k_bst_rank(const uint64_t* __restrict__ bk, const uint32_t* __restrict__ bi, uint64_t m,
                           const uint64_t* __restrict__ ak, const uint32_t* __restrict__ ai, uint64_t n,
                           uint32_t* __restrict__ posb, uint32_t* __restrict__ hist) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = bk[j];
        const uint32_t i = bi[j];
        uint64_t lo = 0, hi = n;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (pair_lt(ak[mid], ai[mid], k, i)) lo = mid + 1;
            else hi = mid;
        }
        posb[j] = (uint32_t)lo;
        atomicAdd(hist + lo, 1u);
    }
}

// Merge, step 2: scatter both sequences. Old entry i goes to i + (new
// entries placed at or before i) = i + incl[i]; new entry j to posb[j] + j.
template <int D>
__global__ void k_bst_scatter(const uint64_t* __restrict__ ak, const uint32_t* __restrict__ ai,
                              const uint32_t* __restrict__ ap, uint64_t n, const uint32_t* __restrict__ excl,
                              const uint32_t* __restrict__ hist, const uint64_t* __restrict__ bk,
                              const uint32_t* __restrict__ bi, const uint32_t* __restrict__ bp, uint64_t m,
                              const uint32_t* __restrict__ posb, uint64_t* __restrict__ ok, uint32_t* __restrict__ oi,
                              uint32_t* __restrict__ op) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n + m; i += stride) {
        uint64_t dst;
        uint64_t k;
        uint32_t id;
        const uint32_t* p;
        if (i < n) {
            dst = i + excl[i] + hist[i];
            k = ak[i];
            id = ai[i];
            p = ap + i * D;
        } else {
            const uint64_t j = i - n;
            dst = posb[j] + j;
            k = bk[j];
            id = bi[j];
            p = bp + j * D;
        }
        ok[dst] = k;
        oi[dst] = id;
#pragma unroll
        for (int d = 0; d < D; ++d) op[dst * D + d] = p[d];
    }
}

// Delete, step 1: claim live ids (alive word 1 -> 0); count them.
__global__ void k_bst_kill(const uint32_t* __restrict__ ids, uint64_t m, uint32_t next_id,
                           uint32_t* __restrict__ alive, unsigned long long* __restrict__ nd) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t id = ids[j];
        if (id < next_id && atomicExch(alive + id, 0u) == 1u) atomicAdd(nd, 1ull);
    }
}

__global__ void k_bst_keep(const uint32_t* __restrict__ ids, uint64_t n, const uint32_t* __restrict__ alive,
                           uint32_t* __restrict__ keep) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        keep[i] = alive[ids[i]];
}

template <int D>
__global__ void k_bst_compact(const uint64_t* __restrict__ ak, const uint32_t* __restrict__ ai,
                              const uint32_t* __restrict__ ap, uint64_t n, const uint32_t* __restrict__ keep,
                              const uint32_t* __restrict__ pos, uint64_t* __restrict__ ok, uint32_t* __restrict__ oi,
                              uint32_t* __restrict__ op) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        if (!keep[i]) continue;
        const uint64_t dst = pos[i];
        ok[dst] = ak[i];
        oi[dst] = ai[i];
#pragma unroll
        for (int d = 0; d < D; ++d) op[dst * D + d] = ap[i * D + d];
    }
}

__global__ void k_bst_fill(uint32_t* __restrict__ p, uint64_t a, uint64_t b, uint32_t v) {
    for (uint64_t i = a + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_bst_iota(uint32_t* __restrict__ p, uint64_t m, uint32_t base) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = base + (uint32_t)i;
}

// ----------------------------------------------------------------- queries
template <int D>
__device__ __forceinline__ uint64_t bst_box_dist(const uint32_t* q, const NodeRec& r) {
    uint64_t s = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const uint32_t x = q[d] < r.lo[d] ? r.lo[d] - q[d] : (q[d] > r.hi[d] ? q[d] - r.hi[d] : 0u);
        s += (uint64_t)x * x;
    }
    return r.cnt ? s : PAD_D2;
}

constexpr int BST_STACK = 48;  // > the deepest tree (about 32 levels)
constexpr int BST_THREADS = 128;

// kNN, a lane per query (k <= 16): seeded with the phi entries on each side
// of the query's own place in key order, then a depth-first walk that
// visits the nearer child first, prunes boxes farther than the k-th
// distance, tests each interior node's pivot point and scans leaves; the
// seeded run is skipped there. The stack of pending nodes is in LDS.
template <int D, int K>
__global__ __launch_bounds__(BST_THREADS) void k_bst_knn(BstView t, uint32_t phi, const uint32_t* __restrict__ qp,
                                                         const uint64_t* __restrict__ qkeys, uint64_t nq,
                                                         const uint32_t* __restrict__ order,
                                                         uint32_t* __restrict__ out_ids, uint64_t* __restrict__ out_d2) {
    __shared__ uint32_t s_stk[BST_STACK][BST_THREADS];
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
    auto take = [&](uint32_t i) {
        uint32_t p[D];
#pragma unroll
        for (int d = 0; d < D; ++d) p[d] = t.pts[(uint64_t)i * D + d];
        const uint64_t dd = pt_dist<D>(q, p);
        if (dd <= bd[K - 1]) {
            const uint32_t id = t.ids[i];
            if (pair_less(dd, id, bd[K - 1], bi[K - 1])) topk_insert<K>(bd, bi, dd, id);
        }
    };
    if (t.n > 0) {
        const uint64_t key = qkeys[qi];
        uint32_t lo = 0, hi = t.n;  // first entry with a key above the query's
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (t.keys[mid] <= key) lo = mid + 1;
            else hi = mid;
        }
        const uint32_t sa = lo > phi ? lo - phi : 0u, sb = min(lo + phi, t.n);
        for (uint32_t i = sa; i < sb; ++i) take(i);
        uint32_t* stk = &s_stk[0][threadIdx.x];
        int sp = 0;
        stk[0] = 0;
        sp = 1;
        while (sp > 0) {
            const uint32_t v = stk[(--sp) * BST_THREADS];
            const NodeRec r = t.node[v];
            if (r.cnt == 0 || bst_box_dist<D>(q, r) > bd[K - 1]) continue;
            const uint2 ab = t.range[v];
            if (r.slot == 1) {
                for (uint32_t i = ab.x; i < ab.y; ++i)
                    if (i < sa || i >= sb) take(i);
                continue;
            }
            const uint32_t m = ab.x + (ab.y - ab.x) / 2;
            if (m < sa || m >= sb) take(m);
            const uint64_t c0 = 2ull * v + 1, c1 = c0 + 1;
            const uint64_t d0 = bst_box_dist<D>(q, t.node[c0]), d1 = bst_box_dist<D>(q, t.node[c1]);
            // push the farther first so the nearer is taken next
            const uint32_t fa = (uint32_t)(d0 <= d1 ? c1 : c0), ne = (uint32_t)(d0 <= d1 ? c0 : c1);
            const uint64_t dfa = d0 <= d1 ? d1 : d0, dne = d0 <= d1 ? d0 : d1;
            if (dfa <= bd[K - 1] && sp < BST_STACK) stk[(sp++) * BST_THREADS] = fa;
            if (dne <= bd[K - 1] && sp < BST_STACK) stk[(sp++) * BST_THREADS] = ne;
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        out_ids[qi * K + j] = bi[j];
        out_d2[qi * K + j] = bd[j];
    }
}

template <int D>
__device__ __forceinline__ int bst_rel(const NodeRec& r, const uint32_t* lo, const uint32_t* hi) {
    if (!r.cnt) return 0;
    bool inside = true;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (r.hi[d] < lo[d] || r.lo[d] > hi[d]) return 0;
        inside = inside && lo[d] <= r.lo[d] && r.hi[d] <= hi[d];
    }
    return inside ? 2 : 1;
}

// Range count (REPORT = false) or report, a lane per box. A subtree inside
// the box counts its size, or reports its run of ids; a straddling leaf is
// scanned; a straddling interior node tests its pivot and goes on into its
// children.
template <int D, bool REPORT>
__global__ __launch_bounds__(BST_THREADS) void k_bst_range(BstView t, const uint32_t* __restrict__ boxes, uint64_t nb,
                                                           const uint32_t* __restrict__ order,
                                                           uint64_t* __restrict__ counts,
                                                           const uint64_t* __restrict__ offsets,
                                                           uint32_t* __restrict__ out) {
    __shared__ uint32_t s_stk[BST_STACK][BST_THREADS];
    const uint64_t tb = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tb >= nb) return;
    const uint64_t b = order ? order[tb] : tb;
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
    auto in_box = [&](uint32_t i) {
        bool in = true;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const uint32_t c = t.pts[(uint64_t)i * D + d];
            in = in && lo[d] <= c && c <= hi[d];
        }
        return in;
    };
    if (!empty && t.n > 0) {
        uint32_t* stk = &s_stk[0][threadIdx.x];
        int sp = 1;
        stk[0] = 0;
        while (sp > 0) {
            const uint32_t v = stk[(--sp) * BST_THREADS];
            const NodeRec r = t.node[v];
            const int rel = bst_rel<D>(r, lo, hi);
            if (rel == 0) continue;
            const uint2 ab = t.range[v];
            if (rel == 2) {
                if (!REPORT) cnt += ab.y - ab.x;
                else
                    for (uint32_t i = ab.x; i < ab.y && o < lim; ++i) out[o++] = t.ids[i];
                continue;
            }
            if (r.slot == 1) {
                for (uint32_t i = ab.x; i < ab.y; ++i)
                    if (in_box(i)) {
                        if (!REPORT) ++cnt;
                        else if (o < lim) out[o++] = t.ids[i];
                    }
                continue;
            }
            const uint32_t m = ab.x + (ab.y - ab.x) / 2;
            if (in_box(m)) {
                if (!REPORT) ++cnt;
                else if (o < lim) out[o++] = t.ids[m];
            }
            if (sp + 2 <= BST_STACK) {
                stk[(sp++) * BST_THREADS] = 2 * v + 2;
                stk[(sp++) * BST_THREADS] = 2 * v + 1;
            }
        }
    }
    if (!REPORT) counts[b] = cnt;
}

}  // namespace
}  // namespace psi

using namespace psi;

struct psi_bst_s {
    psi_index ix = nullptr;  // stream, encode and sort workspace, query ordering, error word
    uint32_t D = 3, curve = 1, phi = 40;
    uint64_t n = 0, H = 0;
    uint32_t depth = 0, next_id = 0;
    Buf keys[2], ids[2], pts[2];
    int cur = 0;
    Buf node, range, alive, bpts, posb, hist, excl, tmp, nd;

    BstView view() const {
        BstView v{};
        v.node = node.as<NodeRec>();
        v.range = range.as<uint2>();
        v.pts = pts[cur].as<uint32_t>();
        v.ids = ids[cur].as<uint32_t>();
        v.keys = keys[cur].as<uint64_t>();
        v.n = (uint32_t)n;
        v.depth = depth;
        return v;
    }
};

namespace {

// Heap depth of BuildSorted's shape over n entries: the first depth whose
// largest range (n halved, rounded down, per level) fits a leaf.
uint32_t bst_depth(uint64_t n, uint32_t phi) {
    uint32_t d = 0;
    for (uint64_t s = n; s > phi; s /= 2) ++d;
    return d;
}

psi_status bst_layout(psi_bst t) {
    hipStream_t st = t->ix->st;
    psi_status s;
    t->depth = bst_depth(t->n, t->phi);
    t->H = (2ull << t->depth) - 1;
    if ((s = t->node.ensure(t->H * sizeof(NodeRec))) != PSI_OK) return s;
    if ((s = t->range.ensure(t->H * 8)) != PSI_OK) return s;
    const unsigned g = blocks_of(t->H, 256);
    if (t->D == 2)
        hipLaunchKernelGGL(k_bst_layout<2>, dim3(g), dim3(256), 0, st, (uint32_t)t->n, t->phi, t->H,
                           t->node.as<NodeRec>(), t->range.as<uint2>(), t->pts[t->cur].as<uint32_t>());
    else
        hipLaunchKernelGGL(k_bst_layout<3>, dim3(g), dim3(256), 0, st, (uint32_t)t->n, t->phi, t->H,
                           t->node.as<NodeRec>(), t->range.as<uint2>(), t->pts[t->cur].as<uint32_t>());
    for (int d = (int)t->depth - 1; d >= 0; --d) {
        const unsigned gi = blocks_of(1ull << d, 256);
        if (t->D == 2)
            hipLaunchKernelGGL(k_bst_inner<2>, dim3(gi), dim3(256), 0, st, (uint32_t)d, t->node.as<NodeRec>(),
                               t->range.as<uint2>(), t->pts[t->cur].as<uint32_t>());
        else
            hipLaunchKernelGGL(k_bst_inner<3>, dim3(gi), dim3(256), 0, st, (uint32_t)d, t->node.as<NodeRec>(),
                               t->range.as<uint2>(), t->pts[t->cur].as<uint32_t>());
    }
    return hip_ok(hipGetLastError());
}

psi_status bst_sorted_arrays(psi_bst t, int b, uint64_t n) {
    psi_status s;
    if ((s = t->keys[b].ensure(std::max<uint64_t>(n, 1) * 8)) != PSI_OK) return s;
    if ((s = t->ids[b].ensure(std::max<uint64_t>(n, 1) * 4)) != PSI_OK) return s;
    return t->pts[b].ensure(std::max<uint64_t>(n, 1) * 4 * t->D);
}

void bst_gather(psi_bst t, const uint32_t* ids, uint64_t n, const uint32_t* src, uint32_t id_base, uint32_t* out) {
    if (!n) return;
    const unsigned g = blocks_of(n, 256);
    if (t->D == 2) hipLaunchKernelGGL(k_bst_gather<2>, dim3(g), dim3(256), 0, t->ix->st, ids, n, src, id_base, out);
    else hipLaunchKernelGGL(k_bst_gather<3>, dim3(g), dim3(256), 0, t->ix->st, ids, n, src, id_base, out);
}

// One word per id handed out (1 = live), grown with its contents kept.
psi_status bst_alive(psi_bst t, uint64_t upto) {
    return t->alive.grow_keep(std::max<uint64_t>(upto, 1) * 4, t->alive.bytes, t->ix->st);
}

}  // namespace

extern "C" {

psi_status psi_bst_create(uint32_t dim, uint32_t curve, uint32_t leaf_wrap, void* hip_stream, psi_bst* out) {
    if (!out || (dim != 2 && dim != 3) || curve > 1 || leaf_wrap < 1 || leaf_wrap > 1024) return PSI_E_ARG;
    *out = nullptr;
    psi_params p{};
    p.dim = dim;
    p.curve = curve;
    p.leaf_size = 32;
    p.fanout = 8;
    p.flags = 0;
    psi_bst t = new (std::nothrow) psi_bst_s;
    if (!t) return PSI_E_NOMEM;
    t->D = dim;
    t->curve = curve;
    t->phi = leaf_wrap;
    psi_status s = psi_create(&p, hip_stream, &t->ix);
    if (s != PSI_OK) {
        delete t;
        return s;
    }
    *out = t;
    return PSI_OK;
}

psi_status psi_bst_destroy(psi_bst t) {
    if (!t) return PSI_E_ARG;
    (void)hipStreamSynchronize(t->ix->st);
    psi_destroy(t->ix);
    delete t;
    return PSI_OK;
}

psi_status psi_bst_build(psi_bst t, const uint32_t* d_pts, uint64_t n) {
    if (!t || (n && !d_pts)) return PSI_E_ARG;
    if (n >= (1ull << 31)) return PSI_E_CAPACITY;
    if (capturing(t->ix->st)) return PSI_E_STATE;
    psi_status s = psi_sync(t->ix);
    if (s != PSI_OK) return s;
    t->n = 0;
    t->cur = 0;
    if ((s = bst_sorted_arrays(t, 0, n)) != PSI_OK) return s;
    if ((s = bst_alive(t, n)) != PSI_OK) return s;
    if (n) {
        int w = 0;
        if ((s = t->keys[1].ensure(n * 8)) != PSI_OK) return s;  // the keys in input order (scratch)
        if ((s = encode_sort(t->ix, d_pts, n, t->keys[1].as<uint64_t>(), 0, &w)) != PSI_OK) return s;
        Sorter& S = t->ix->sorter;
        hipStream_t st = t->ix->st;
        if ((s = hip_ok(hipMemcpyAsync(t->keys[0].p, S.k[w].p, n * 8, hipMemcpyDeviceToDevice, st))) != PSI_OK) return s;
        if ((s = hip_ok(hipMemcpyAsync(t->ids[0].p, S.i[w].p, n * 4, hipMemcpyDeviceToDevice, st))) != PSI_OK) return s;
        bst_gather(t, t->ids[0].as<uint32_t>(), n, d_pts, 0, t->pts[0].as<uint32_t>());
        hipLaunchKernelGGL(k_bst_fill, dim3(blocks_of(n, 256)), dim3(256), 0, st, t->alive.as<uint32_t>(), 0ull, n,
                           1u);
    }
    t->n = n;
    t->next_id = (uint32_t)n;
    if ((s = bst_layout(t)) != PSI_OK) return s;
    return psi_sync(t->ix);
}

psi_status psi_bst_batch_insert(psi_bst t, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids) {
    if (!t || (m && (!d_pts || !d_new_ids))) return PSI_E_ARG;
    if (m == 0) return PSI_OK;
    if ((uint64_t)t->next_id + m >= (1ull << 31)) return PSI_E_CAPACITY;
    if (capturing(t->ix->st)) return PSI_E_STATE;
    psi_status s;
    hipStream_t st = t->ix->st;
    const uint64_t n = t->n;
    const uint32_t base = t->next_id;
    if ((s = t->bpts.ensure(m * 4 * t->D)) != PSI_OK) return s;
    if ((s = t->posb.ensure(m * 4)) != PSI_OK) return s;
    if ((s = t->hist.ensure((n + 1) * 4)) != PSI_OK) return s;
    if ((s = t->excl.ensure((n + 2) * 4)) != PSI_OK) return s;
    if ((s = t->tmp.ensure((scan_tmp_words(n + 1) + 8) * 4)) != PSI_OK) return s;
    if ((s = bst_alive(t, (uint64_t)base + m)) != PSI_OK) return s;
    const int o = t->cur ^ 1;
    if ((s = bst_sorted_arrays(t, o, n + m)) != PSI_OK) return s;
    // the batch's sorted pairs (ids base .. base + m - 1) and their points
    int w = 0;
    if ((s = t->keys[o].ensure((n + m) * 8)) != PSI_OK) return s;
    if ((s = encode_sort(t->ix, d_pts, m, t->keys[o].as<uint64_t>(), base, &w)) != PSI_OK) return s;
    Sorter& S = t->ix->sorter;
    const uint64_t* bk = S.k[w].as<uint64_t>();
    const uint32_t* bi = S.i[w].as<uint32_t>();
    bst_gather(t, bi, m, d_pts, base, t->bpts.as<uint32_t>());
    // place of every new entry, shift of every old one, scatter
    launch_fill_u32(st, t->hist.as<uint32_t>(), n + 1, 0u);
    hipLaunchKernelGGL(k_bst_rank, dim3(blocks_of(m, 256)), dim3(256), 0, st, bk, bi, m, t->keys[t->cur].as<uint64_t>(),
                       t->ids[t->cur].as<uint32_t>(), n, t->posb.as<uint32_t>(), t->hist.as<uint32_t>());
    launch_scan_u32(st, t->hist.as<uint32_t>(), t->excl.as<uint32_t>(), n + 1, t->excl.as<uint32_t>() + n + 1,
                    t->tmp.as<uint32_t>());
    const unsigned g = blocks_of(n + m, 256);
#define PSI_BS(DD)                                                                                                   \
    hipLaunchKernelGGL(k_bst_scatter<DD>, dim3(g), dim3(256), 0, st, t->keys[t->cur].as<uint64_t>(),                  \
                       t->ids[t->cur].as<uint32_t>(), t->pts[t->cur].as<uint32_t>(), n, t->excl.as<uint32_t>(),      \
                       t->hist.as<uint32_t>(), bk, bi, t->bpts.as<uint32_t>(), m, t->posb.as<uint32_t>(),           \
                       t->keys[o].as<uint64_t>(), t->ids[o].as<uint32_t>(), t->pts[o].as<uint32_t>())
    if (t->D == 2) PSI_BS(2);
    else PSI_BS(3);
#undef PSI_BS
    hipLaunchKernelGGL(k_bst_fill, dim3(blocks_of(m, 256)), dim3(256), 0, st, t->alive.as<uint32_t>(), (uint64_t)base,
                       (uint64_t)base + m, 1u);
    // the new ids in input order: base + i
    hipLaunchKernelGGL(k_bst_iota, dim3(blocks_of(m, 256)), dim3(256), 0, st, d_new_ids, m, base);
    t->cur = o;
    t->n = n + m;
    t->next_id = base + (uint32_t)m;
    if ((s = bst_layout(t)) != PSI_OK) return s;
    return psi_sync(t->ix);
}

psi_status psi_bst_batch_delete(psi_bst t, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted) {
    if (!t || (m && !d_ids)) return PSI_E_ARG;
    if (capturing(t->ix->st)) return PSI_E_STATE;
    psi_status s;
    hipStream_t st = t->ix->st;
    const uint64_t n = t->n;
    if ((s = t->nd.ensure(8)) != PSI_OK) return s;
    launch_fill_u32(st, t->nd.as<uint32_t>(), 2, 0u);
    if (m)
        hipLaunchKernelGGL(k_bst_kill, dim3(blocks_of(m, 256)), dim3(256), 0, st, d_ids, m, t->next_id,
                           t->alive.as<uint32_t>(), t->nd.as<unsigned long long>());
    uint64_t removed = 0;
    if ((s = hip_ok(hipMemcpyAsync(&removed, t->nd.p, 8, hipMemcpyDeviceToHost, st))) != PSI_OK) return s;
    if ((s = hip_ok(hipStreamSynchronize(st))) != PSI_OK) return s;
    if (d_ndeleted &&
        (s = hip_ok(hipMemcpyAsync(d_ndeleted, t->nd.p, 8, hipMemcpyDeviceToDevice, st))) != PSI_OK)
        return s;
    if (removed) {
        const int o = t->cur ^ 1;
        if ((s = bst_sorted_arrays(t, o, n)) != PSI_OK) return s;
        if ((s = t->hist.ensure((n + 1) * 4)) != PSI_OK) return s;
        if ((s = t->excl.ensure((n + 2) * 4)) != PSI_OK) return s;
        if ((s = t->tmp.ensure((scan_tmp_words(n) + 8) * 4)) != PSI_OK) return s;
        hipLaunchKernelGGL(k_bst_keep, dim3(blocks_of(n, 256)), dim3(256), 0, st, t->ids[t->cur].as<uint32_t>(), n,
                           t->alive.as<uint32_t>(), t->hist.as<uint32_t>());
        launch_scan_u32(st, t->hist.as<uint32_t>(), t->excl.as<uint32_t>(), n, t->excl.as<uint32_t>() + n,
                        t->tmp.as<uint32_t>());
        const unsigned g = blocks_of(n, 256);
#define PSI_BC(DD)                                                                                                  \
    hipLaunchKernelGGL(k_bst_compact<DD>, dim3(g), dim3(256), 0, st, t->keys[t->cur].as<uint64_t>(),                \
                       t->ids[t->cur].as<uint32_t>(), t->pts[t->cur].as<uint32_t>(), n, t->hist.as<uint32_t>(),    \
                       t->excl.as<uint32_t>(), t->keys[o].as<uint64_t>(), t->ids[o].as<uint32_t>(),                \
                       t->pts[o].as<uint32_t>())
        if (t->D == 2) PSI_BC(2);
        else PSI_BC(3);
#undef PSI_BC
        t->cur = o;
        t->n = n - removed;
        if ((s = bst_layout(t)) != PSI_OK) return s;
    }
    return psi_sync(t->ix);
}

psi_status psi_bst_knn(psi_bst t, const uint32_t* d_q, uint64_t nq, uint32_t k, uint32_t* d_ids, uint64_t* d_d2) {
    if (!t || k == 0 || k > 16 || (nq && (!d_q || !d_ids || !d_d2))) return PSI_E_ARG;
    if (nq == 0) return PSI_OK;
    const uint32_t* order = nullptr;
    psi_status s = query_order(t->ix, d_q, nq, false, &order);  // also the queries' curve keys
    if (s != PSI_OK) return s;
    const BstView v = t->view();
    const unsigned g = (unsigned)((nq + BST_THREADS - 1) / BST_THREADS);
    const uint64_t* qk = t->ix->qkeys.as<uint64_t>();
    hipStream_t st = t->ix->st;
#define PSI_BK(DD, KK) hipLaunchKernelGGL((k_bst_knn<DD, KK>), dim3(g), dim3(BST_THREADS), 0, st, v, t->phi, d_q, qk, nq, order, d_ids, d_d2)
#define PSI_BK_ALL(DD)                                                                                       \
    switch (k) {                                                                                             \
        case 1: PSI_BK(DD, 1); break;   case 2: PSI_BK(DD, 2); break;   case 3: PSI_BK(DD, 3); break;        \
        case 4: PSI_BK(DD, 4); break;   case 5: PSI_BK(DD, 5); break;   case 6: PSI_BK(DD, 6); break;        \
        case 7: PSI_BK(DD, 7); break;   case 8: PSI_BK(DD, 8); break;   case 9: PSI_BK(DD, 9); break;        \
        case 10: PSI_BK(DD, 10); break; case 11: PSI_BK(DD, 11); break; case 12: PSI_BK(DD, 12); break;      \
        case 13: PSI_BK(DD, 13); break; case 14: PSI_BK(DD, 14); break; case 15: PSI_BK(DD, 15); break;      \
        default: PSI_BK(DD, 16); break;                                                                      \
    }
    if (t->D == 2) { PSI_BK_ALL(2) } else { PSI_BK_ALL(3) }
#undef PSI_BK_ALL
#undef PSI_BK
    return hip_ok(hipGetLastError());
}

static psi_status bst_range(psi_bst t, const uint32_t* d_boxes, uint64_t nb, uint64_t* d_counts,
                            const uint64_t* d_offsets, uint32_t* d_ids, bool report) {
    const uint32_t* order = nullptr;
    psi_status s = query_order(t->ix, d_boxes, nb, true, &order);
    if (s != PSI_OK) return s;
    const BstView v = t->view();
    const unsigned g = (unsigned)((nb + BST_THREADS - 1) / BST_THREADS);
    hipStream_t st = t->ix->st;
    if (t->D == 2) {
        if (report) hipLaunchKernelGGL((k_bst_range<2, true>), dim3(g), dim3(BST_THREADS), 0, st, v, d_boxes, nb, order, nullptr, d_offsets, d_ids);
        else hipLaunchKernelGGL((k_bst_range<2, false>), dim3(g), dim3(BST_THREADS), 0, st, v, d_boxes, nb, order, d_counts, nullptr, nullptr);
    } else {
        if (report) hipLaunchKernelGGL((k_bst_range<3, true>), dim3(g), dim3(BST_THREADS), 0, st, v, d_boxes, nb, order, nullptr, d_offsets, d_ids);
        else hipLaunchKernelGGL((k_bst_range<3, false>), dim3(g), dim3(BST_THREADS), 0, st, v, d_boxes, nb, order, d_counts, nullptr, nullptr);
    }
    return hip_ok(hipGetLastError());
}

psi_status psi_bst_range_count(psi_bst t, const uint32_t* d_boxes, uint64_t nb, uint64_t* d_counts) {
    if (!t || (nb && (!d_boxes || !d_counts))) return PSI_E_ARG;
    if (nb == 0) return PSI_OK;
    return bst_range(t, d_boxes, nb, d_counts, nullptr, nullptr, false);
}

psi_status psi_bst_range_report(psi_bst t, const uint32_t* d_boxes, uint64_t nb, const uint64_t* d_offsets,
                                uint32_t* d_ids) {
    if (!t || (nb && (!d_boxes || !d_offsets))) return PSI_E_ARG;
    if (nb == 0) return PSI_OK;
    return bst_range(t, d_boxes, nb, nullptr, d_offsets, d_ids, true);
}

psi_status psi_bst_sync(psi_bst t) {
    if (!t) return PSI_E_ARG;
    return psi_sync(t->ix);
}

psi_status psi_bst_shape(psi_bst t, uint64_t* h_n, uint32_t* h_depth, uint64_t* h_heap) {
    if (!t || !h_n || !h_depth || !h_heap) return PSI_E_ARG;
    psi_status s = psi_sync(t->ix);
    if (s != PSI_OK) return s;
    *h_n = t->n;
    *h_depth = t->depth;
    *h_heap = t->H;
    return PSI_OK;
}

psi_status psi_bst_export(psi_bst t, uint32_t* d_nodes, uint32_t* d_ranges, uint32_t* d_ids, uint32_t* d_pts) {
    if (!t || !d_nodes || !d_ranges || !d_ids || !d_pts) return PSI_E_ARG;
    hipStream_t st = t->ix->st;
    psi_status s;
    if (t->H &&
        ((s = hip_ok(hipMemcpyAsync(d_nodes, t->node.p, t->H * sizeof(NodeRec), hipMemcpyDeviceToDevice, st))) != PSI_OK ||
         (s = hip_ok(hipMemcpyAsync(d_ranges, t->range.p, t->H * 8, hipMemcpyDeviceToDevice, st))) != PSI_OK))
        return s;
    if (t->n &&
        ((s = hip_ok(hipMemcpyAsync(d_ids, t->ids[t->cur].p, t->n * 4, hipMemcpyDeviceToDevice, st))) != PSI_OK ||
         (s = hip_ok(hipMemcpyAsync(d_pts, t->pts[t->cur].p, t->n * 4 * t->D, hipMemcpyDeviceToDevice, st))) != PSI_OK))
        return s;
    return psi_sync(t->ix);
}

}  // extern "C"
