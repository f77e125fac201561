// kNN and range queries over the SPaC-tree (Sec. 2.2 definitions; the
// traversal follows App. C: visit subtrees in increasing distance from the
// query to their boxes and prune a box farther than the current k-th
// neighbour; leaves are scanned in full because their order is relaxed).
//
// The tree is implicit (node i of a level has children B i .. B i + B - 1).
// The seeded kNN walks (lane per query and wave per query) and the range
// walk keep a stack of child masks in LDS, one word per level: expanding a
// node tests all its children at once and remembers the ones still to
// visit. The nearest-child-first kNN (lane per query) keeps no stack: after
// finishing a node it re-scores the siblings from the parent and moves to the
// nearest one not yet visited.
//
// Exactness: a subtree is skipped only when its box distance is strictly
// greater than the k-th distance, so an equal-distance point with a smaller
// id can still enter the result.
#include "psi_hilbert.h"
#include "psi_kern.h"

namespace psi {

namespace {

inline unsigned blocks_for(uint64_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

template <int D>
__device__ __forceinline__ uint64_t box_dist(const uint32_t* q, const NodeRec& r) {
    uint64_t s = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const uint32_t a = q[d] < r.lo[d] ? r.lo[d] - q[d] : 0u;
        const uint32_t b = q[d] > r.hi[d] ? q[d] - r.hi[d] : 0u;
        const uint64_t x = a | b;
        s += x * x;
    }
    return r.cnt ? s : PAD_D2;
}

__device__ __forceinline__ NodeRec fetch(const TreeView& t, const LevelInfo* lv, uint32_t l, uint64_t i) {
    return l == t.h ? t.leaf[i] : t.inner[lv[l].off + i];
}

// ------------------------------------------------------- kNN, lane per query
template <int D, int K>
__global__ __launch_bounds__(256) void k_knn_lane(TreeView tv, const uint32_t* __restrict__ qp, uint64_t nq,
                                                  const uint32_t* __restrict__ order,
                                                  uint32_t* __restrict__ out_ids, uint64_t* __restrict__ out_d2) {
    __shared__ LevelInfo s_lv[MAX_LEVELS];
    const TreeView t = resolve_tree(tv);
    if (threadIdx.x <= t.h) s_lv[threadIdx.x] = tv.dt->lv[threadIdx.x];
    __syncthreads();
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
    if (t.L > 0) {
        const uint32_t C = t.C;
        uint32_t l = 0;
        uint64_t i = 0;
        bool down = true;
        for (;;) {
            if (down) {
                if (l == t.h) {
                    const NodeRec r = t.leaf[i];
                    const uint32_t* s = t.slots + (uint64_t)r.slot * (D + 1) * C;
                    for (uint32_t e = 0; e < r.cnt; e += 4) {
                        uint4 X[D];
#pragma unroll
                        for (int d = 0; d < D; ++d) X[d] = *reinterpret_cast<const uint4*>(s + d * C + e);
                        const uint4 I = *reinterpret_cast<const uint4*>(s + D * C + e);
                        const uint32_t xs[4][3] = {{X[0].x, X[1].x, D == 3 ? X[D - 1].x : 0u},
                                                   {X[0].y, X[1].y, D == 3 ? X[D - 1].y : 0u},
                                                   {X[0].z, X[1].z, D == 3 ? X[D - 1].z : 0u},
                                                   {X[0].w, X[1].w, D == 3 ? X[D - 1].w : 0u}};
                        const uint32_t is[4] = {I.x, I.y, I.z, I.w};
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (e + u < r.cnt) {
                                const uint64_t dd = pt_dist<D>(q, xs[u]);
                                if (pair_less(dd, is[u], bd[K - 1], bi[K - 1])) topk_insert<K>(bd, bi, dd, is[u]);
                            }
                        }
                    }
                    down = false;
                    continue;
                }
                const uint64_t c0 = i * t.B, c1 = min<uint64_t>(c0 + t.B, s_lv[l + 1].n);
                uint64_t best = PAD_D2, bc = c0;
                for (uint64_t c = c0; c < c1; ++c) {
                    const uint64_t dd = box_dist<D>(q, fetch(t, s_lv, l + 1, c));
                    if (dd < best) {
                        best = dd;
                        bc = c;
                    }
                }
                if (best != PAD_D2 && best <= bd[K - 1]) {
                    ++l;
                    i = bc;
                } else {
                    down = false;
                }
            } else {
                if (l == 0) break;
                const uint64_t p = i / t.B, s0 = p * t.B, s1 = min<uint64_t>(s0 + t.B, s_lv[l].n);
                const uint64_t dcur = box_dist<D>(q, fetch(t, s_lv, l, i));
                uint64_t best = PAD_D2, bs = 0;
                bool found = false;
                for (uint64_t s = s0; s < s1; ++s) {
                    if (s == i) continue;
                    const uint64_t dd = box_dist<D>(q, fetch(t, s_lv, l, s));
                    const bool after = dd > dcur || (dd == dcur && s > i);
                    if (after && (!found || dd < best)) {
                        best = dd;
                        bs = s;
                        found = true;
                    }
                }
                if (found && best != PAD_D2 && best <= bd[K - 1]) {
                    i = bs;
                    down = true;
                } else {
                    --l;
                    i = p;
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        out_ids[qi * K + j] = bi[j];
        out_d2[qi * K + j] = bd[j];
    }
}

// ---------------------------------------- kNN, lane per query, seeded search
// The query's own curve key locates the leaf whose key range holds it (a
// binary search over the leaf pivots); that leaf and its two neighbours in
// curve order seed the k best with nearby points. The tree is then walked
// depth first in fixed child order, skipping every box farther than the
// current k-th distance and the seed leaves already scanned. A good seed
// radius makes this visit little more than the leaves the final k-th
// distance ball touches, without re-scoring siblings.
//
// Seed leaves, where most entries enter the k best, are scanned in one
// pass: four entries at a time (coordinates and ids together), each one
// inserted straight from registers when it beats the current k-th pair.
//
// Leaves met by the walk, where few entries do, are scanned in two passes,
// 64 entries at a time: the distances of all entries (coordinates only)
// against the k-th distance at the start give a bit mask of candidates; the
// candidates, two at a time, are read again (both loads in flight together)
// and inserted. The lanes of a wave then go through the insertion code about
// as often as the lane with the most candidates, not once for every entry
// that any lane inserts.
template <int D, int K>
__device__ __forceinline__ void scan_seed_leaf(const TreeView& t, uint32_t slot, uint32_t cnt, const uint32_t* q,
                                               uint64_t (&bd)[K], uint32_t (&bi)[K]) {
    const uint32_t C = t.C;
    const uint32_t* s = t.slots + (uint64_t)slot * (D + 1) * C;
    for (uint32_t e = 0; e < cnt; e += 4) {
        uint4 X[D];
#pragma unroll
        for (int d = 0; d < D; ++d) X[d] = *reinterpret_cast<const uint4*>(s + d * C + e);
        const uint4 I = *reinterpret_cast<const uint4*>(s + D * C + e);
        const uint32_t xs[4][3] = {{X[0].x, X[1].x, D == 3 ? X[D - 1].x : 0u},
                                   {X[0].y, X[1].y, D == 3 ? X[D - 1].y : 0u},
                                   {X[0].z, X[1].z, D == 3 ? X[D - 1].z : 0u},
                                   {X[0].w, X[1].w, D == 3 ? X[D - 1].w : 0u}};
        uint64_t dd[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) dd[u] = pt_dist<D>(q, xs[u]);
        const uint32_t nu = min(cnt - e, 4u);
#pragma unroll 1
        for (uint32_t u = 0; u < nu; ++u) {
            const uint64_t d = u == 0 ? dd[0] : (u == 1 ? dd[1] : (u == 2 ? dd[2] : dd[3]));
            const uint32_t id = u == 0 ? I.x : (u == 1 ? I.y : (u == 2 ? I.z : I.w));
            if (pair_less(d, id, bd[K - 1], bi[K - 1])) topk_insert<K>(bd, bi, d, id);
        }
    }
}

template <int D, int K>
__device__ __forceinline__ void scan_leaf(const TreeView& t, uint32_t slot, uint32_t cnt, const uint32_t* q,
                                          uint64_t (&bd)[K], uint32_t (&bi)[K]) {
    const uint32_t C = t.C;
    const uint32_t* s = t.slots + (uint64_t)slot * (D + 1) * C;
    for (uint32_t e0 = 0; e0 < cnt; e0 += 64) {
        const uint32_t ce = min(cnt - e0, 64u);
        const uint64_t kth = bd[K - 1];
        uint64_t cm = 0;
        for (uint32_t e = 0; e < ce; e += 4) {
            uint4 X[D];
#pragma unroll
            for (int d = 0; d < D; ++d) X[d] = *reinterpret_cast<const uint4*>(s + d * C + e0 + e);
            const uint32_t xs[4][3] = {{X[0].x, X[1].x, D == 3 ? X[D - 1].x : 0u},
                                       {X[0].y, X[1].y, D == 3 ? X[D - 1].y : 0u},
                                       {X[0].z, X[1].z, D == 3 ? X[D - 1].z : 0u},
                                       {X[0].w, X[1].w, D == 3 ? X[D - 1].w : 0u}};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool c = e + u < ce && pt_dist<D>(q, xs[u]) <= kth;
                cm |= c ? 1ull << (e + u) : 0ull;
            }
        }
        while (cm) {
            const uint32_t ea = e0 + (uint32_t)__builtin_ctzll(cm);
            cm &= cm - 1;
            const bool two = cm != 0;
            const uint32_t eb = two ? e0 + (uint32_t)__builtin_ctzll(cm) : ea;
            if (two) cm &= cm - 1;
            uint32_t pa[D], pb[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                pa[d] = s[d * C + ea];
                pb[d] = s[d * C + eb];
            }
            const uint32_t ia = s[D * C + ea], ib = s[D * C + eb];
            const uint64_t da = pt_dist<D>(q, pa);
            if (pair_less(da, ia, bd[K - 1], bi[K - 1])) topk_insert<K>(bd, bi, da, ia);
            const uint64_t db = pt_dist<D>(q, pb);
            if (two && pair_less(db, ib, bd[K - 1], bi[K - 1])) topk_insert<K>(bd, bi, db, ib);
        }
    }
}

// Seeded search over any tree exposed through an accessor `T` with
// L(), h(), B(), levn(l) (nodes of level l), dist(l, i, q) (squared distance
// from q to the box of node i of level l, the leaves being level h; PAD_D2
// for an empty node), leaf_sc(i) (slot and count of leaf i) and pkey(i).
template <int D, int K, class T>
__device__ __forceinline__ void knn_seeded(const T& tr, const TreeView& tv, const uint32_t* q, uint64_t key,
                                           uint64_t (&bd)[K], uint32_t (&bi)[K]) {
    const uint32_t L = tr.L();
    if (L == 0) return;
    uint32_t lo = 0, hi = L;  // first pivot key above the query's key
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (tr.pkey(mid) <= key) lo = mid + 1;
        else hi = mid;
    }
    const uint32_t j = lo ? lo - 1 : 0u;
    const uint32_t ja = j ? j - 1 : 0u, jb = min(j + 1, L - 1);
    for (uint32_t x = ja; x <= jb; ++x) {
        const uint2 sc = tr.leaf_sc(x);  // (count, slot)
        scan_seed_leaf<D, K>(tv, sc.y, sc.x, q, bd, bi);
    }
    const uint32_t B = tr.B(), h = tr.h();
    uint32_t l = 0, i = 0;
    for (;;) {
        const uint64_t bdist = tr.dist(l, i, q);
        bool descend = false;
        if (bdist != PAD_D2 && bdist <= bd[K - 1]) {
            if (l == h) {
                if (i < ja || i > jb) {
                    const uint2 sc = tr.leaf_sc(i);
                    scan_leaf<D, K>(tv, sc.y, sc.x, q, bd, bi);
                }
            } else {
                descend = true;
            }
        }
        if (descend) {
            ++l;
            i *= B;
            continue;
        }
        bool done = false;
        for (;;) {
            if (l == 0) {
                done = true;
                break;
            }
            if ((i + 1) % B != 0 && i + 1 < tr.levn(l)) {
                ++i;
                break;
            }
            --l;
            i /= B;
        }
        if (done) break;
    }
}

// What one search touched: box tests (a node's box read and compared),
// leaves scanned and points scanned (seed leaves included).
struct WalkCount {
    uint32_t boxes = 0, leaves = 0, points = 0;
};

// Sum over the wave (every lane takes part).
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int o = 32; o >= 1; o >>= 1) v += shfl_u32(v, (int)(lane_id() ^ (uint32_t)o));
    return v;
}

// Adds a wave's query count and walk counts to stats[0..3] (lane 0).
__device__ __forceinline__ void add_walk_stats(unsigned long long* stats, uint32_t queries, const WalkCount& wc) {
    const uint32_t a = wave_sum_u32(queries), b = wave_sum_u32(wc.boxes), c = wave_sum_u32(wc.leaves),
                   d = wave_sum_u32(wc.points);
    if (lane_id() == 0) {
        atomicAdd(stats + 0, (unsigned long long)a);
        atomicAdd(stats + 1, (unsigned long long)b);
        atomicAdd(stats + 2, (unsigned long long)c);
        atomicAdd(stats + 3, (unsigned long long)d);
    }
}

// The same search in three phases, so that the lanes of a wave run the same
// code at the same time (the search is bound by instruction issue, and a
// wave whose lanes split between expanding nodes and scanning leaves pays
// for both): (1) the seed leaves are scanned; (2) the tree is walked with a
// stack of child masks, one per level, in LDS (`stk`): expanding a node
// reads the boxes of all its children in one batch of independent loads and
// keeps those within the current k-th distance; children that are leaves go
// to a list of candidate leaves in LDS (`cand`, ncap entries) instead of
// being scanned; (3) the candidates are scanned, each checked again against
// the k-th distance of the moment. A full list is scanned (and emptied)
// before more leaves go in, so any number of candidates is handled. Both LDS
// arrays hold one word per lane per entry, `stride` words apart. Needs
// h() <= the stack depth; the caller takes the other walk beyond it.
// sr: seed radius (the leaves j - sr .. j + sr around the query's own leaf j
// seed the search); ncap: candidate leaves collected before a scan
// (<= the LDS list's length).
template <int D, int K, class T>
__device__ __forceinline__ void knn_seeded_masks(const T& tr, const TreeView& tv, const uint32_t* q, uint64_t key,
                                                 uint64_t (&bd)[K], uint32_t (&bi)[K], uint32_t* __restrict__ stk,
                                                 uint32_t* __restrict__ cand, uint32_t stride, uint32_t sr,
                                                 uint32_t ncap, WalkCount& wc) {
    const uint32_t L = tr.L();
    if (L == 0) return;
    uint32_t lo = 0, hi = L;  // first pivot key above the query's key
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (tr.pkey(mid) <= key) lo = mid + 1;
        else hi = mid;
    }
    const uint32_t j = lo ? lo - 1 : 0u;
    const uint32_t ja = j > sr ? j - sr : 0u, jb = min(j + sr, L - 1);
    for (uint32_t x = ja; x <= jb; ++x) {
        const uint2 sc = tr.leaf_sc(x);  // (count, slot)
        scan_seed_leaf<D, K>(tv, sc.y, sc.x, q, bd, bi);
        wc.leaves += 1;
        wc.points += sc.x;
    }
    const uint32_t B = tr.B(), h = tr.h();
    if (h == 0) return;  // a single leaf, scanned as a seed
    // children of `node` on level l + 1 within the k-th distance (the seed
    // leaves left out)
    auto expand = [&](uint32_t l, uint32_t node) -> uint32_t {
        const uint32_t c0 = node * B, nc = min(B, tr.levn(l + 1) - c0);
        const uint64_t kth = bd[K - 1];
        const bool leaves = l + 1 == h;
        uint32_t m = 0;
        for (uint32_t x0 = 0; x0 < nc; x0 += 8) {
            uint64_t d[8];
            tr.dist8(l + 1, c0 + x0, min(nc - x0, 8u), q, d);
#pragma unroll
            for (uint32_t u = 0; u < 8; ++u) {
                const uint32_t c = c0 + x0 + u;
                const bool keep = x0 + u < nc && d[u] != PAD_D2 && d[u] <= kth && !(leaves && c >= ja && c <= jb);
                m |= keep ? 1u << (x0 + u) : 0u;
            }
        }
        wc.boxes += nc;
        return m;
    };
    {
        const uint64_t d = tr.dist(0, 0, q);
        wc.boxes += 1;
        if (d == PAD_D2 || d > bd[K - 1]) return;
    }
    // walk state: the masks on the stack cover inner nodes only (level l's
    // mask covers the children base .. base + B - 1 on level l + 1 < h);
    // pend: leaf children (from pbase) not yet on the candidate list
    uint32_t l = 0, base = 0, pend = 0, pbase = 0, ncand = 0;
    bool walking = h > 1;
    const uint32_t m0 = expand(0, 0);
    if (walking) stk[0] = m0;
    else pend = m0;
    for (;;) {
        // (2) fill the candidate list. Every pass of the loop ends in one
        // expansion (the costly step, run by the whole wave at once); the
        // cheap steps before it (moving pending leaves to the list, popping
        // exhausted levels) run in loops of their own, so a lane busy with
        // them does not hold the others' expansions back a pass each.
        while (ncand < ncap) {
            while (pend && ncand < ncap) {
                const uint32_t b = (uint32_t)__builtin_ctz(pend);
                pend &= pend - 1;
                cand[ncand * stride] = pbase + b;
                ++ncand;
            }
            if (pend || !walking) break;
            uint32_t m = stk[l * stride];
            while (m == 0 && l > 0) {
                --l;
                base = base / B / B * B;
                m = stk[l * stride];
            }
            if (m == 0) {
                walking = false;
                break;
            }
            const uint32_t b = (uint32_t)__builtin_ctz(m);
            stk[l * stride] = m & (m - 1);
            // (a node farther than the k-th distance has all its children
            // farther too: expanding it finds none, no separate check)
            const uint32_t c = base + b;
            const uint32_t cm = expand(l + 1, c);
            if (cm == 0) continue;
            if (l + 2 == h) {  // c's children are leaves
                pend = cm;
                pbase = c * B;
                continue;
            }
            ++l;
            stk[l * stride] = cm;
            base = c * B;
        }
        // (3) scan the candidates
        for (uint32_t x = 0; x < ncand; ++x) {
            const uint32_t c = cand[x * stride];
            const uint64_t d = tr.dist(h, c, q);
            const uint2 sc = tr.leaf_sc(c);
            wc.boxes += 1;
            if (d <= bd[K - 1]) {
                scan_leaf<D, K>(tv, sc.y, sc.x, q, bd, bi);
                wc.leaves += 1;
                wc.points += sc.x;
            }
        }
        ncand = 0;
        if (!walking && pend == 0) break;
    }
}

// Squared distance from q to a packed box (PAD_D2 for an empty node). No
// branch: the box is decoded whether or not it is empty, so a caller's
// loads of several boxes stay independent and go out together.
template <int D>
__device__ __forceinline__ uint64_t packed_dist(const uint32_t* q, uint4 v) {
    const uint64_t a = ((uint64_t)v.y << 32) | v.x, b = ((uint64_t)v.w << 32) | v.z;
    constexpr int W = BoxBits<D>::W;
    constexpr uint64_t M = (1ull << W) - 1;
    uint64_t s = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const uint32_t lo = (uint32_t)((a >> (d * W)) & M), hi = (uint32_t)((b >> (d * W)) & M);
        const uint32_t x = q[d] < lo ? lo - q[d] : (q[d] > hi ? q[d] - hi : 0u);
        s += (uint64_t)x * x;
    }
    return (a >> 63) ? PAD_D2 : s;
}

// Accessor of a single index whose level table sits in LDS: box tests read
// the packed boxes, leaf scans the slot and count of the leaf record.
template <int D>
struct SingleTree {
    const TreeView& t;
    const LevelInfo* lv;
    __device__ uint32_t L() const { return (uint32_t)t.L; }
    __device__ uint32_t h() const { return t.h; }
    __device__ uint32_t B() const { return t.B; }
    __device__ uint32_t levn(uint32_t l) const { return (uint32_t)lv[l].n; }
    __device__ uint64_t dist(uint32_t l, uint32_t i, const uint32_t* q) const {
        return packed_dist<D>(q, l == t.h ? t.cleaf[i] : t.cinner[lv[l].off + i]);
    }
    // distances of nodes c .. c + n - 1 (1 <= n <= 8) of level l into d[0..n);
    // the eight loads are unconditional (clamped to the last node) and go
    // out together
    __device__ void dist8(uint32_t l, uint32_t c, uint32_t n, const uint32_t* q, uint64_t (&d)[8]) const {
        const uint4* p = (l == t.h ? t.cleaf : t.cinner + lv[l].off) + c;
        uint4 v[8];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) v[u] = p[min(u, n - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u) d[u] = packed_dist<D>(q, v[u]);
    }
    __device__ uint2 leaf_sc(uint32_t i) const { return *reinterpret_cast<const uint2*>(&t.leaf[i].cnt); }
    __device__ uint64_t pkey(uint32_t i) const { return t.pkey[i]; }
};

// The same over the node records themselves (boxes unpacked: more bytes,
// less arithmetic per box test; the wave-per-query search, where one box
// test serves a whole wave's lane, gains from it).
template <int D>
struct SingleTreeRec : SingleTree<D> {
    __device__ uint64_t dist(uint32_t l, uint32_t i, const uint32_t* q) const {
        return box_dist<D>(q, l == this->t.h ? this->t.leaf[i] : this->t.inner[this->lv[l].off + i]);
    }
};

// MASKS: the three-phase walk; s_stk (dynamic LDS) holds its stack of child
// masks, hcap levels of one word per lane, then ncap candidate-leaf
// words per lane; a taller tree (never met: hcap bounds the
// height of every tree the buffers can hold) leaves its queries unanswered
// and flags ERR_STACK. stats (nullable, MASKS only): the walk counts are
// added to stats[0..3] (queries, box tests, leaves, points).
template <int D, int K, bool MASKS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((K <= 8 || K == 10) ? 5 : 1))) void k_knn_seed(TreeView tv, const uint32_t* __restrict__ qp,
                                                  const uint64_t* __restrict__ qkeys, uint64_t nq,
                                                  const uint32_t* __restrict__ order, uint32_t hcap,
                                                  uint32_t sr, uint32_t ncap,
                                                  uint32_t* __restrict__ err, unsigned long long* __restrict__ stats,
                                                  uint32_t* __restrict__ out_ids, uint64_t* __restrict__ out_d2) {
    __shared__ LevelInfo s_lv[MAX_LEVELS];
    extern __shared__ uint32_t s_stk[];
    const TreeView t = resolve_tree(tv);
    if (threadIdx.x <= t.h) s_lv[threadIdx.x] = tv.dt->lv[threadIdx.x];
    __syncthreads();
    const uint64_t tq = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    WalkCount wc;
    if (tq < nq) {
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
        const SingleTree<D> tr{t, s_lv};
        if (!MASKS) knn_seeded<D, K>(tr, t, q, qkeys[qi], bd, bi);
        else if (t.h <= hcap)
            knn_seeded_masks<D, K>(tr, t, q, qkeys[qi], bd, bi, s_stk + threadIdx.x,
                                   s_stk + (size_t)hcap * blockDim.x + threadIdx.x, blockDim.x, sr, ncap, wc);
        else if (tq == 0) atomicOr(err, ERR_STACK);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            out_ids[qi * K + j] = bi[j];
            out_d2[qi * K + j] = bd[j];
        }
    }
    if (MASKS && stats) add_walk_stats(stats, tq < nq ? 1u : 0u, wc);
}

// ---------------------------------------------- kNN over many small indexes
// Accessor of index m among a batch of indexes sharing global arrays.
template <int D>
struct MultiTree {
    const IdxMeta* m;
    const NodeRec* inner;
    const NodeRec* leafs;
    const uint64_t* pk;
    uint32_t b;
    __device__ uint32_t L() const { return m->L; }
    __device__ uint32_t h() const { return m->h; }
    __device__ uint32_t B() const { return b; }
    __device__ uint32_t levn(uint32_t l) const { return m->lvl_n[l]; }
    __device__ NodeRec node(uint32_t l, uint32_t i) const { return inner[m->inner_base + m->lvl_off[l] + i]; }
    __device__ NodeRec leaf(uint32_t i) const { return leafs[m->leaf_base + i]; }
    __device__ uint64_t dist(uint32_t l, uint32_t i, const uint32_t* q) const {
        return box_dist<D>(q, l == m->h ? leaf(i) : node(l, i));
    }
    // as SingleTree::dist8, over the node records, four loads at a time
    __device__ void dist8(uint32_t l, uint32_t c, uint32_t n, const uint32_t* q, uint64_t (&d)[8]) const {
        const NodeRec* p = (l == m->h ? leafs + m->leaf_base : inner + m->inner_base + m->lvl_off[l]) + c;
#pragma unroll
        for (uint32_t h4 = 0; h4 < 8; h4 += 4) {
            NodeRec r[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) r[u] = p[min(h4 + u, n - 1)];
#pragma unroll
            for (int u = 0; u < 4; ++u) d[h4 + u] = box_dist<D>(q, r[u]);
        }
    }
    __device__ uint2 leaf_sc(uint32_t i) const {
        const NodeRec r = leaf(i);
        return make_uint2(r.cnt, r.slot);
    }
    __device__ uint64_t pkey(uint32_t i) const { return pk[m->leaf_base + i]; }
};

__global__ void k_chunk_counts(const uint64_t* __restrict__ q_off, uint32_t num, uint32_t* __restrict__ cnt) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < num) cnt[s] = (uint32_t)((q_off[s + 1] - q_off[s] + 63) / 64);
}

// Persistent: every wave takes (index, 64-query chunk) items from an atomic
// counter until none are left, so uneven batches spread over the whole GPU.
// s_stk: the walk's stacks of child masks, hcap (the tallest index's
// height) levels of one word per lane, then KNN_CAND candidate-leaf words
// per lane.
template <int D, int CURVE, int K>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((D == 2 && K <= 4) ? 5 : 1))) void k_multi_knn(TreeView tv, const IdxMeta* __restrict__ meta, uint32_t num,
                                                   const uint64_t* __restrict__ q_off, const uint32_t* __restrict__ qp,
                                                   const uint32_t* __restrict__ pref, uint32_t* __restrict__ work_ctr,
                                                   uint32_t hcap, uint32_t* __restrict__ out_ids,
                                                   uint64_t* __restrict__ out_d2, uint32_t* __restrict__ err) {
    extern __shared__ uint32_t s_stk[];
    const uint32_t lane = lane_id();
    const uint32_t W = pref[num];
    for (;;) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(work_ctr, 1u);
        item = shfl_u32(item, 0);
        if (item >= W) break;
        uint32_t lo = 0, hi = num;  // index of the item: largest s with pref[s] <= item
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pref[mid] <= item) lo = mid;
            else hi = mid;
        }
        const uint32_t s = lo;
        const uint64_t qb = q_off[s] + (uint64_t)(item - pref[s]) * 64;
        const uint64_t qe = min<uint64_t>(qb + 64, q_off[s + 1]);
        const uint64_t qi = qb + lane;
        if (qi < qe) {
            uint32_t q[D];
#pragma unroll
            for (int d = 0; d < D; ++d) q[d] = qp[qi * D + d];
            if (!coord_ok<D>(q)) atomicOr(err, ERR_RANGE);
            uint64_t bd[K];
            uint32_t bi[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                bd[j] = PAD_D2;
                bi[j] = PAD_ID;
            }
            const MultiTree<D> tr{meta + s, tv.inner, tv.leaf, tv.pkey, tv.B};
            WalkCount wc;
            if (tr.h() <= hcap)
                knn_seeded_masks<D, K>(tr, tv, q, sfc_key_tab<D, CURVE>(q), bd, bi, s_stk + threadIdx.x,
                                       s_stk + (size_t)hcap * blockDim.x + threadIdx.x, blockDim.x, 1u,
                                       KNN_CAND, wc);
            else atomicOr(err, ERR_STACK);
#pragma unroll
            for (int j = 0; j < K; ++j) {
                out_ids[qi * K + j] = bi[j];
                out_d2[qi * K + j] = bd[j];
            }
        }
    }
}

// ------------------------------------------------------- kNN, wave per query
// For k > 16. The k best pairs live in LDS, ascending, in two copies (a merge
// writes the other one). A leaf is merged in one entry per lane: the entries
// that beat the current k-th pair are ranked among themselves, and every
// list entry and candidate finds its new place by binary search in the other
// sequence. The search is seeded with the leaves around the query's curve
// position until they hold at least max(2k, 64) points; the tree is then
// walked as in the lane-per-query search, with the wave testing a node's
// children one per lane and the stack of child masks in LDS.
constexpr int KW_WAVES = 4;

template <int KMAX>
struct KList {
    uint64_t (*d)[KMAX];  // [2][KMAX]
    uint32_t (*i)[KMAX];
    uint64_t* cd;         // [64] candidates
    uint32_t* ci;
};

// Merges entries e0 .. min(cnt, e0 + 64) - 1 of the leaf stored at `s`.
template <int D, int KMAX>
__device__ __forceinline__ void kw_merge64(const KList<KMAX>& Ls, int& cur, uint32_t k, const uint32_t* s,
                                           uint32_t C, uint32_t e0, uint32_t cnt, const uint32_t* q) {
    const uint32_t lane = lane_id();
    const uint32_t e = e0 + lane;
    uint64_t dd = PAD_D2;
    uint32_t id = PAD_ID;
    bool cand = false;
    if (e < cnt) {
        uint32_t p[D];
#pragma unroll
        for (int d = 0; d < D; ++d) p[d] = s[d * C + e];
        dd = pt_dist<D>(q, p);
        if (dd <= Ls.d[cur][k - 1]) {
            id = s[D * C + e];
            cand = pair_less(dd, id, Ls.d[cur][k - 1], Ls.i[cur][k - 1]);
        }
    }
    const uint64_t cm = ballot(cand);
    if (cm == 0) return;
    const uint32_t nc = (uint32_t)__popcll(cm);
    if (cand) {
        const uint32_t slot_c = count_below(cm);
        Ls.cd[slot_c] = dd;
        Ls.ci[slot_c] = id;
    }
    __builtin_amdgcn_wave_barrier();
    uint32_t cpos = 0, rank = 0;
    if (cand) {
        for (uint32_t x = 0; x < nc; ++x) rank += pair_less(Ls.cd[x], Ls.ci[x], dd, id) ? 1u : 0u;
        uint32_t lo = 0, hi = k;  // list entries below the candidate
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pair_less(Ls.d[cur][mid], Ls.i[cur][mid], dd, id)) lo = mid + 1;
            else hi = mid;
        }
        cpos = rank + lo;
    }
    __builtin_amdgcn_wave_barrier();  // every lane has read the unsorted candidates
    if (cand) {
        Ls.cd[rank] = dd;
        Ls.ci[rank] = id;
    }
    __builtin_amdgcn_wave_barrier();
    const int nxt = cur ^ 1;
    for (uint32_t x = lane; x < k; x += 64) {
        const uint64_t ld = Ls.d[cur][x];
        const uint32_t li = Ls.i[cur][x];
        uint32_t lo = 0, hi = nc;  // candidates below list entry x
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pair_less(Ls.cd[mid], Ls.ci[mid], ld, li)) lo = mid + 1;
            else hi = mid;
        }
        if (x + lo < k) {
            Ls.d[nxt][x + lo] = ld;
            Ls.i[nxt][x + lo] = li;
        }
    }
    if (cand && cpos < k) {
        Ls.d[nxt][cpos] = dd;
        Ls.i[nxt][cpos] = id;
    }
    __builtin_amdgcn_wave_barrier();
    cur = nxt;
}

// Merges the leaf with the given slot and count, 64 entries at a time.
template <int D, int KMAX>
__device__ __forceinline__ void kw_merge_leaf(const KList<KMAX>& Ls, int& cur, uint32_t k, const TreeView& t,
                                              uint32_t slot, uint32_t cnt, const uint32_t* q) {
    const uint32_t* s = t.slots + (uint64_t)slot * (D + 1) * t.C;
    for (uint32_t e0 = 0; e0 < cnt; e0 += 64) kw_merge64<D, KMAX>(Ls, cur, k, s, t.C, e0, cnt, q);
}

// stats (nullable): as for k_knn_seed.
template <int D, int KMAX>
__global__ __launch_bounds__(256) void k_knn_wave(TreeView tv, const uint32_t* __restrict__ qp,
                                                  const uint64_t* __restrict__ qkeys, uint64_t nq,
                                                  const uint32_t* __restrict__ order, uint32_t k,
                                                  unsigned long long* __restrict__ stats,
                                                  uint32_t* __restrict__ out_ids, uint64_t* __restrict__ out_d2) {
    __shared__ LevelInfo s_lv[MAX_LEVELS];
    __shared__ uint64_t s_d[KW_WAVES][2][KMAX];
    __shared__ uint32_t s_i[KW_WAVES][2][KMAX];
    __shared__ uint64_t s_cd[KW_WAVES][64];
    __shared__ uint32_t s_ci[KW_WAVES][64];
    __shared__ uint32_t s_mask[KW_WAVES][MAX_LEVELS];
    const TreeView t = resolve_tree(tv);
    if (threadIdx.x <= t.h) s_lv[threadIdx.x] = tv.dt->lv[threadIdx.x];
    __syncthreads();
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = lane_id();
    const uint64_t tq = (uint64_t)blockIdx.x * KW_WAVES + w;
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
    const KList<KMAX> Ls{s_d[w], s_i[w], s_cd[w], s_ci[w]};
    int cur = 0;
    const SingleTreeRec<D> tr{{t, s_lv}};
    const uint32_t L = (uint32_t)t.L;
    uint32_t n_box = 0, n_leaf = 0, n_pts = 0;  // wave-uniform walk counts
    if (L > 0) {
        // seed leaves: outward from the leaf holding the query's key
        const uint64_t key = qkeys[qi];
        uint32_t lo = 0, hi = L;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (tr.pkey(mid) <= key) lo = mid + 1;
            else hi = mid;
        }
        const uint32_t j = lo ? lo - 1 : 0u;
        const uint32_t want = max(2 * k, 64u);
        uint32_t ja = j, jb = j, have = tr.leaf_sc(j).x;
        while (have < want && (ja > 0 || jb + 1 < L)) {
            if (ja > 0) have += tr.leaf_sc(--ja).x;
            if (jb + 1 < L) have += tr.leaf_sc(++jb).x;
        }
        for (uint32_t x = ja; x <= jb; ++x) {
            const uint2 sc = tr.leaf_sc(x);
            kw_merge_leaf<D, KMAX>(Ls, cur, k, t, sc.y, sc.x, q);
            n_leaf += 1;
            n_pts += sc.x;
        }
        const uint32_t B = t.B, h = t.h;
        // children of `node` (level l) within the k-th distance, seeds left out
        auto expand = [&](uint32_t l, uint32_t node) -> uint32_t {
            const uint32_t c0 = node * B, nc = min(B, tr.levn(l + 1) - c0);
            const uint64_t kth = s_d[w][cur][k - 1];
            const uint32_t c = c0 + lane;
            bool keep = false;
            if (lane < nc) {
                const uint64_t d = tr.dist(l + 1, c, q);
                keep = d != PAD_D2 && d <= kth && !(l + 1 == h && c >= ja && c <= jb);
            }
            n_box += nc;
            return (uint32_t)ballot(keep);
        };
        const uint64_t droot = tr.dist(0, 0, q);
        n_box += 1;
        if (h > 0 && droot != PAD_D2 && droot <= s_d[w][cur][k - 1]) {
            uint32_t l = 0, base = 0;
            uint32_t m0 = expand(0, 0);
            if (lane == 0) s_mask[w][0] = m0;
            __builtin_amdgcn_wave_barrier();
            for (;;) {
                const uint32_t m = s_mask[w][l];
                if (m == 0) {
                    if (l == 0) break;
                    --l;
                    base = base / B / B * B;
                    continue;
                }
                const uint32_t b = (uint32_t)__builtin_ctz(m);
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) s_mask[w][l] = m & (m - 1);
                __builtin_amdgcn_wave_barrier();
                const uint32_t c = base + b;
                const uint64_t d = tr.dist(l + 1, c, q);
                n_box += 1;
                if (d > s_d[w][cur][k - 1]) continue;
                if (l + 1 == h) {
                    const uint2 sc = tr.leaf_sc(c);
                    kw_merge_leaf<D, KMAX>(Ls, cur, k, t, sc.y, sc.x, q);
                    n_leaf += 1;
                    n_pts += sc.x;
                    continue;
                }
                const uint32_t cm = expand(l + 1, c);
                if (cm == 0) continue;
                ++l;
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) s_mask[w][l] = cm;
                __builtin_amdgcn_wave_barrier();
                base = c * B;
            }
        }
    }
    for (uint32_t x = lane; x < k; x += 64) {
        out_ids[qi * k + x] = s_i[w][cur][x];
        out_d2[qi * k + x] = s_d[w][cur][x];
    }
    if (stats && lane == 0) {
        atomicAdd(stats + 0, 1ull);
        atomicAdd(stats + 1, (unsigned long long)n_box);
        atomicAdd(stats + 2, (unsigned long long)n_leaf);
        atomicAdd(stats + 3, (unsigned long long)n_pts);
    }
}

// ------------------------------------------------------------ range queries
template <int D>
__device__ __forceinline__ int box_relation(const NodeRec& r, const uint32_t* lo, const uint32_t* hi) {
    bool inside = true;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (r.hi[d] < lo[d] || r.lo[d] > hi[d]) return 0;  // disjoint
        inside = inside && lo[d] <= r.lo[d] && r.hi[d] <= hi[d];
    }
    return inside ? 2 : 1;
}

template <int D>
__device__ __forceinline__ bool in_box(const uint32_t* p, const uint32_t* lo, const uint32_t* hi) {
    bool in = true;
#pragma unroll
    for (int d = 0; d < D; ++d) in = in && lo[d] <= p[d] && p[d] <= hi[d];
    return in;
}

// REPORT = false: count; REPORT = true: write ids to out[0 .. lim).
template <int D, bool REPORT>
__global__ __launch_bounds__(256) void k_range(TreeView tv, const uint32_t* __restrict__ boxes, uint64_t nb,
                                               uint64_t* __restrict__ counts, const uint64_t* __restrict__ offsets,
                                               uint32_t* __restrict__ out_ids) {
    __shared__ LevelInfo s_lv[MAX_LEVELS];
    const TreeView t = resolve_tree(tv);
    if (threadIdx.x <= t.h) s_lv[threadIdx.x] = tv.dt->lv[threadIdx.x];
    __syncthreads();
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    uint32_t lo[D], hi[D];
    bool empty = false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = boxes[b * 2 * D + d];
        hi[d] = boxes[b * 2 * D + D + d];
        empty = empty || lo[d] > hi[d];
    }
    uint64_t cnt = 0;
    uint64_t o = 0, lim = 0;
    uint32_t* out = nullptr;
    if (REPORT) {
        o = offsets[b];
        lim = offsets[b + 1];
        out = out_ids;
    }
    const uint32_t C = t.C;
    if (!empty && t.L > 0) {
        uint32_t l = 0;
        uint64_t i = 0;
        for (;;) {
            const NodeRec r = fetch(t, s_lv, l, i);
            const int rel = r.cnt ? box_relation<D>(r, lo, hi) : 0;
            bool descend = false;
            if (rel == 2) {
                if (!REPORT) {
                    cnt += r.cnt;
                } else {
                    const uint64_t span = s_lv[l].span;
                    const uint64_t j1 = min<uint64_t>((i + 1) * span, t.L);
                    for (uint64_t j = i * span; j < j1; ++j) {
                        const NodeRec lf = t.leaf[j];
                        const uint32_t* s = t.slots + (uint64_t)lf.slot * (D + 1) * C + D * C;
                        for (uint32_t e = 0; e < lf.cnt && o < lim; ++e) out[o++] = s[e];
                    }
                }
            } else if (rel == 1) {
                if (l == t.h) {
                    const uint32_t* s = t.slots + (uint64_t)r.slot * (D + 1) * C;
                    for (uint32_t e = 0; e < r.cnt; ++e) {
                        uint32_t p[D];
#pragma unroll
                        for (int d = 0; d < D; ++d) p[d] = s[d * C + e];
                        if (in_box<D>(p, lo, hi)) {
                            if (!REPORT) ++cnt;
                            else if (o < lim) out[o++] = s[D * C + e];
                        }
                    }
                } else {
                    descend = true;
                }
            }
            if (descend) {
                ++l;
                i *= t.B;
                continue;
            }
            bool done = false;
            for (;;) {
                if (l == 0) {
                    done = true;
                    break;
                }
                if ((i + 1) % t.B != 0 && i + 1 < s_lv[l].n) {
                    ++i;
                    break;
                }
                --l;
                i /= t.B;
            }
            if (done) break;
        }
    }
    if (!REPORT) counts[b] = cnt;
}

// ------------------------------------------------- range queries, wave per box
// One wave per box. Expanding a node tests all its children at once (one
// lane per child); children that straddle the box are remembered in a
// per-level mask (a stack of masks in LDS) and expanded depth first. Leaves
// that straddle the box are scanned two at a time, one per half-wave and one
// entry per lane; whole subtrees inside the box add their counts, or, for
// reports, have their leaves' ids copied two leaves at a time.
constexpr int RW_WAVES = 4;
constexpr int RW_PAIRS = 4;  // straddling leaf pairs whose first rows are loaded together

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t* total) {
    const uint32_t lane = lane_id();
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = shfl_u32(x, (int)lane - o);
        if (lane >= (uint32_t)o) x += y;
    }
    *total = shfl_u32(x, 63);
    return x - v;
}

// Copies the ids of the leaves held by the lanes in `m` (lane x: count lc,
// exclusive output position pos, slot) to out[o + pos ..], two leaves at a
// time, one per half-wave, so that every store is two contiguous runs.
// All lanes of the wave take part.
template <int D>
__device__ __forceinline__ void copy_leaf_ids(const TreeView& t, uint64_t m, uint32_t lc, uint32_t pos, uint32_t slot,
                                              uint64_t o, uint64_t lim, uint32_t* __restrict__ out) {
    const uint32_t lane = lane_id(), hl = lane & 31u;
    while (m) {
        const uint32_t xa = (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        uint32_t xb = 64u;  // no second leaf
        if (m) {
            xb = (uint32_t)__builtin_ctzll(m);
            m &= m - 1;
        }
        const uint32_t mine = lane < 32u ? xa : xb;
        const uint32_t c0 = shfl_u32(lc, (int)(mine & 63u)), p0 = shfl_u32(pos, (int)(mine & 63u)),
                       s0 = shfl_u32(slot, (int)(mine & 63u));
        const uint32_t cx = mine < 64u ? c0 : 0u;
        const uint32_t* s = t.slots + (uint64_t)s0 * (D + 1) * t.C + D * t.C;
        for (uint32_t e = hl; e < cx; e += 32) {
            const uint64_t dst = o + p0 + e;
            if (dst < lim) out[dst] = s[e];
        }
    }
}

template <int D, bool REPORT>
__global__ __launch_bounds__(256) void k_range_wave(TreeView tv, const uint32_t* __restrict__ boxes, uint64_t nb,
                                                    const uint32_t* __restrict__ order,
                                                    uint64_t* __restrict__ counts,
                                                    const uint64_t* __restrict__ offsets,
                                                    uint32_t* __restrict__ out) {
    __shared__ LevelInfo s_lv[MAX_LEVELS];
    __shared__ uint64_t s_mask[RW_WAVES][MAX_LEVELS];
    __shared__ uint64_t s_base[RW_WAVES][MAX_LEVELS];
    const TreeView t = resolve_tree(tv);
    if (threadIdx.x <= t.h) s_lv[threadIdx.x] = tv.dt->lv[threadIdx.x];
    __syncthreads();
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = lane_id();
    const uint64_t bx = (uint64_t)blockIdx.x * RW_WAVES + w;
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
    uint64_t cnt = 0;
    uint64_t o = 0, lim = 0;
    if (REPORT) {
        o = offsets[b];
        lim = offsets[b + 1];
    }
    const uint32_t C = t.C, B = t.B, h = t.h;

    // Visit nc children starting at c0 on level l (lane c owns child c0 + c);
    // lane c takes part when bit c / B of pm is set (its parent is expanded).
    auto visit = [&](uint32_t l, uint64_t c0, uint32_t nc, uint64_t pm) {
        const bool on = lane < nc && ((pm >> (lane / B)) & 1ull);
        NodeRec r = {};
        int rel = 0;
        if (on) {
            r = fetch(t, s_lv, l, c0 + lane);
            rel = r.cnt ? box_relation<D>(r, lo, hi) : 0;
        }
        const uint64_t inside = ballot(rel == 2);
        const uint64_t partial = ballot(rel == 1);
        if (l < h) {
            s_mask[w][l] = partial;
            s_base[w][l] = c0;
            if (!REPORT) {
                uint32_t tot;
                (void)wave_excl_scan(rel == 2 ? r.cnt : 0u, &tot);
                cnt += tot;
            } else {
                uint64_t m = inside;
                while (m) {  // copy every leaf under each inside child, one leaf per lane
                    const uint32_t c = (uint32_t)__builtin_ctzll(m);
                    m &= m - 1;
                    const uint64_t span = s_lv[l].span;
                    const uint64_t j0 = (c0 + c) * span, j1 = min<uint64_t>(j0 + span, t.L);
                    for (uint64_t jb = j0; jb < j1; jb += 64) {
                        const uint64_t j = jb + lane;
                        const NodeRec lf = j < j1 ? t.leaf[j] : NodeRec{};
                        const uint32_t lc = j < j1 ? lf.cnt : 0u;
                        uint32_t tot;
                        const uint32_t pos = wave_excl_scan(lc, &tot);
                        copy_leaf_ids<D>(t, ballot(lc != 0), lc, pos, lf.slot, o, lim, out);
                        o += tot;
                    }
                }
            }
            return;
        }
        // leaf level: inside leaves, one leaf per lane
        {
            const uint32_t lc = rel == 2 ? r.cnt : 0u;
            uint32_t tot;
            const uint32_t pos = wave_excl_scan(lc, &tot);
            if (REPORT) copy_leaf_ids<D>(t, ballot(lc != 0), lc, pos, r.slot, o, lim, out);
            if (REPORT) o += tot;
            else cnt += tot;
        }
        // straddling leaves: up to RW_PAIRS pairs at a time, a leaf per
        // half-wave (entry e of a leaf on lane e mod 32 of its half); the
        // first 32 entries of every leaf of the batch are loaded together,
        // the rest (leaves grown past 32 by inserts) leaf pair by pair
        uint64_t m = partial;
        const uint32_t hl = lane & 31u;
        while (m) {
            uint32_t rc[RW_PAIRS], rs[RW_PAIRS];
#pragma unroll
            for (int q = 0; q < RW_PAIRS; ++q) {
                uint32_t ca = 64u, cb = 64u;  // 64: no leaf
                if (m) {
                    ca = (uint32_t)__builtin_ctzll(m);
                    m &= m - 1;
                }
                if (m) {
                    cb = (uint32_t)__builtin_ctzll(m);
                    m &= m - 1;
                }
                const uint32_t mine = lane < 32u ? ca : cb;
                const uint32_t sc = shfl_u32(r.cnt, (int)(mine & 63u)), ss = shfl_u32(r.slot, (int)(mine & 63u));
                rc[q] = mine < 64u ? sc : 0u;
                rs[q] = mine < 64u ? ss : 0u;
            }
            uint32_t pc[RW_PAIRS][D];
#pragma unroll
            for (int q = 0; q < RW_PAIRS; ++q) {
                const uint32_t* s = t.slots + (uint64_t)rs[q] * (D + 1) * C;
                const bool on = hl < rc[q];
#pragma unroll
                for (int d = 0; d < D; ++d) pc[q][d] = on ? s[d * C + hl] : 0u;
            }
#pragma unroll
            for (int q = 0; q < RW_PAIRS; ++q) {
                const bool in = hl < rc[q] && in_box<D>(pc[q], lo, hi);
                const uint64_t hit = ballot(in);
                if (REPORT && in) {
                    const uint64_t dst = o + count_below(hit);
                    if (dst < lim) out[dst] = t.slots[(uint64_t)rs[q] * (D + 1) * C + D * C + hl];
                }
                if (REPORT) o += (uint32_t)__popcll(hit);
                else cnt += (uint32_t)__popcll(hit);
            }
#pragma unroll
            for (int q = 0; q < RW_PAIRS; ++q) {
                const uint32_t rmax = max((uint32_t)__builtin_amdgcn_readlane((int)rc[q], 0),
                                          (uint32_t)__builtin_amdgcn_readlane((int)rc[q], 32));
                const uint32_t* s = t.slots + (uint64_t)rs[q] * (D + 1) * C;
                for (uint32_t e0 = 32; e0 < rmax; e0 += 32) {
                    const uint32_t e = e0 + hl;
                    bool in = false;
                    if (e < rc[q]) {
                        uint32_t p[D];
#pragma unroll
                        for (int d = 0; d < D; ++d) p[d] = s[d * C + e];
                        in = in_box<D>(p, lo, hi);
                    }
                    const uint64_t hit = ballot(in);
                    if (REPORT && in) {
                        const uint64_t dst = o + count_below(hit);
                        if (dst < lim) out[dst] = s[D * C + e];
                    }
                    if (REPORT) o += (uint32_t)__popcll(hit);
                    else cnt += (uint32_t)__popcll(hit);
                }
            }
        }
    };

    if (!empty && t.L > 0) {
        visit(0, 0, 1, 1ull);
        // the straddling nodes of one group of G = 64 / B siblings are
        // expanded together: their children fill one wave of lanes
        const uint32_t G = 64u / B;
        const uint64_t gsel = G >= 64u ? ~0ull : (1ull << G) - 1;
        int d = 0;
        while (h > 0 && d >= 0) {
            const uint64_t m = s_mask[w][d];
            if (m == 0) {
                --d;
                continue;
            }
            const uint32_t bit = (uint32_t)__builtin_ctzll(m);
            const uint32_t g0 = bit - bit % G;
            const uint64_t gm = (m >> g0) & gsel;
            s_mask[w][d] = m & ~(gm << g0);
            const uint64_t c0 = (s_base[w][d] + g0) * B;
            const uint32_t nc = (uint32_t)min<uint64_t>((uint64_t)G * B, s_lv[d + 1].n - c0);
            visit((uint32_t)d + 1, c0, nc, gm);
            if ((uint32_t)d + 1 < h) ++d;
        }
    }
    if (!REPORT && lane == 0) counts[b] = cnt;
}

}  // namespace

void launch_knn(hipStream_t st, int dim, const TreeView& t, const uint32_t* q, const uint64_t* qkeys, uint64_t nq,
                const uint32_t* order, uint32_t k, int variant, uint32_t hcap, const KnnTuning& tune,
                uint32_t* err, unsigned long long* stats, uint32_t* ids, uint64_t* d2) {
    if (nq == 0) return;
    const bool masks = hcap <= KNN_STACK_MAX;
    const uint32_t sr = tune.seed_leaves / 2, ncap = max(1u, min(tune.cand, KNN_CAND_MAX));
    const size_t lds = masks ? (size_t)(hcap + ncap) * 256 * 4 : 0;
    const unsigned gl = blocks_for(nq, 256);
    const unsigned gw = blocks_for(nq, KW_WAVES);
#define PSI_KL(D, K)                                                                                             \
    do {                                                                                                         \
        if (variant == 1) hipLaunchKernelGGL((k_knn_lane<D, K>), dim3(gl), dim3(256), 0, st, t, q, nq, order, ids, d2); \
        else if (masks) hipLaunchKernelGGL((k_knn_seed<D, K, true>), dim3(gl), dim3(256), lds, st, t, q, qkeys, nq, order, hcap, sr, ncap, err, stats, ids, d2); \
        else hipLaunchKernelGGL((k_knn_seed<D, K, false>), dim3(gl), dim3(256), 0, st, t, q, qkeys, nq, order, hcap, sr, ncap, err, nullptr, ids, d2); \
    } while (0)
#define PSI_KL_ALL(D)                                                                                    \
    switch (k) {                                                                                         \
        case 1: PSI_KL(D, 1); break;   case 2: PSI_KL(D, 2); break;   case 3: PSI_KL(D, 3); break;       \
        case 4: PSI_KL(D, 4); break;   case 5: PSI_KL(D, 5); break;   case 6: PSI_KL(D, 6); break;       \
        case 7: PSI_KL(D, 7); break;   case 8: PSI_KL(D, 8); break;   case 9: PSI_KL(D, 9); break;       \
        case 10: PSI_KL(D, 10); break; case 11: PSI_KL(D, 11); break; case 12: PSI_KL(D, 12); break;     \
        case 13: PSI_KL(D, 13); break; case 14: PSI_KL(D, 14); break; case 15: PSI_KL(D, 15); break;     \
        case 16: PSI_KL(D, 16); break;                                                                   \
        default:                                                                                         \
            if (k <= 32) hipLaunchKernelGGL((k_knn_wave<D, 32>), dim3(gw), dim3(256), 0, st, t, q, qkeys, nq, order, k, stats, ids, d2); \
            else if (k <= 64) hipLaunchKernelGGL((k_knn_wave<D, 64>), dim3(gw), dim3(256), 0, st, t, q, qkeys, nq, order, k, stats, ids, d2); \
            else hipLaunchKernelGGL((k_knn_wave<D, 128>), dim3(gw), dim3(256), 0, st, t, q, qkeys, nq, order, k, stats, ids, d2); \
    }
    if (dim == 2) { PSI_KL_ALL(2) } else { PSI_KL_ALL(3) }
#undef PSI_KL_ALL
#undef PSI_KL
}

void launch_multi_knn(hipStream_t st, int dim, int curve, const TreeView& tv, const IdxMeta* meta, uint32_t num,
                      const uint64_t* q_off, const uint32_t* q, uint32_t* chunk_pref, uint32_t* work_ctr, uint32_t k,
                      uint32_t hcap, uint32_t* ids, uint64_t* d2, uint32_t* tmp, uint32_t* err) {
    if (num == 0) return;
    hipLaunchKernelGGL(k_chunk_counts, dim3(blocks_for(num, 256)), dim3(256), 0, st, q_off, num, chunk_pref);
    launch_scan_u32(st, chunk_pref, chunk_pref, num, chunk_pref + num, tmp);
    launch_fill_u32(st, work_ctr, 1, 0u);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const dim3 g((unsigned)(cus * 8));
    const size_t lds = (size_t)(hcap + KNN_CAND) * 256 * 4;
#define PSI_MK(D, CV, K) hipLaunchKernelGGL((k_multi_knn<D, CV, K>), g, dim3(256), lds, st, tv, meta, num, q_off, q, chunk_pref, work_ctr, hcap, ids, d2, err)
#define PSI_MK_K(D, CV)                                                                                  \
    switch (k) {                                                                                         \
        case 1: PSI_MK(D, CV, 1); break;  case 2: PSI_MK(D, CV, 2); break;  case 4: PSI_MK(D, CV, 4); break; \
        case 8: PSI_MK(D, CV, 8); break;  case 10: PSI_MK(D, CV, 10); break; case 16: PSI_MK(D, CV, 16); break; \
        default: break;                                                                                  \
    }
    if (dim == 2 && curve == 0) { PSI_MK_K(2, 0) }
    else if (dim == 2) { PSI_MK_K(2, 1) }
    else if (curve == 0) { PSI_MK_K(3, 0) }
    else { PSI_MK_K(3, 1) }
#undef PSI_MK_K
#undef PSI_MK
}

void launch_range_count(hipStream_t st, int dim, const TreeView& t, const uint32_t* boxes, uint64_t nb,
                        const uint32_t* order, uint64_t* counts) {
    if (nb == 0) return;
    const unsigned g = blocks_for(nb, RW_WAVES);
    if (dim == 2) hipLaunchKernelGGL((k_range_wave<2, false>), dim3(g), dim3(256), 0, st, t, boxes, nb, order, counts, nullptr, nullptr);
    else hipLaunchKernelGGL((k_range_wave<3, false>), dim3(g), dim3(256), 0, st, t, boxes, nb, order, counts, nullptr, nullptr);
}

void launch_range_report(hipStream_t st, int dim, const TreeView& t, const uint32_t* boxes, uint64_t nb,
                         const uint32_t* order, const uint64_t* offsets, uint32_t* ids) {
    if (nb == 0) return;
    const unsigned g = blocks_for(nb, RW_WAVES);
    if (dim == 2) hipLaunchKernelGGL((k_range_wave<2, true>), dim3(g), dim3(256), 0, st, t, boxes, nb, order, nullptr, offsets, ids);
    else hipLaunchKernelGGL((k_range_wave<3, true>), dim3(g), dim3(256), 0, st, t, boxes, nb, order, nullptr, offsets, ids);
}

void launch_range_count_lane(hipStream_t st, int dim, const TreeView& t, const uint32_t* boxes, uint64_t nb,
                             uint64_t* counts) {
    if (nb == 0) return;
    const unsigned g = blocks_for(nb, 256);
    if (dim == 2) hipLaunchKernelGGL((k_range<2, false>), dim3(g), dim3(256), 0, st, t, boxes, nb, counts, nullptr, nullptr);
    else hipLaunchKernelGGL((k_range<3, false>), dim3(g), dim3(256), 0, st, t, boxes, nb, counts, nullptr, nullptr);
}

}  // namespace psi
