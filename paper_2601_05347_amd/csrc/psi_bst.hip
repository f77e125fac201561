// The SPaC-tree in the paper's own shape (Sec. 4): a binary search tree on
// (curve key, id) whose subtrees of at most phi points are wrapped into
// leaves, and whose interior nodes each hold one point, the pivot. Builds
// follow Alg. 3's BuildSorted; batch insertions and deletions follow
// Alg. 4's join-based recursion: weight balance (alpha = 0.2) restored by
// Join's rotations, the leaf wrap kept by Node(), and App. C's local
// rebuild of a leaf and its share of the batch below 4 phi points.
//
// Layout: pools of interior nodes (64 B: box, subtree size, pivot key, id
// and point, two child references) and of leaves (32 B: box, count, sorted
// flag; the entries in a slot of phi keys, ids and points). A reference is
// a node index, or a leaf index with the top bit set.
//
// Updates are functional: nothing reachable from the current root is
// written, so a pool that runs out during an update costs a retry (grow the
// pools, run the update again from the same root), never a broken tree. The
// recursion runs level by level:
//  * down, a thread per subtree the batch reaches: an interior node splits
//    its batch range at its pivot and leaves a record of the join to do; a
//    leaf takes its share at once (appended while it fits phi; rebuilt by
//    BuildSorted with the share below 4 phi; exposed and gone on down
//    otherwise; an empty leaf with a large share is rebuilt by the parallel
//    BuildSorted below);
//  * up, level by level from the deepest, a thread per record joins the two
//    updated sides around the pivot (Join2 when a delete removed it); the
//    spine walks, rotations, Expose and Node()'s wrapping run in that thread.
// Every node and leaf an update drops (exposed, flattened into a leaf,
// replaced on the path) is listed and goes to the free lists once the new
// root is committed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/psi.h"
#include "psi_index.h"
#include "psi_kern.h"

namespace psi {
namespace {

inline unsigned blocks_of(uint64_t n, unsigned per) {
    const uint64_t b = (n + per - 1) / per;
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(b, 1u << 20));
}

constexpr uint32_t JB_LEAF = 0x80000000u;  // reference to a leaf
constexpr uint32_t JB_NIL = 0xFFFFFFFFu;
constexpr uint32_t JB_IN = 0x40000000u;    // range walk: a subtree inside the box
constexpr uint32_t JB_PHI_MAX = 64;        // leaf wrap limit (sizes of the per-thread arrays)
constexpr int JB_STACK = 96;               // spine stacks of Join and the largest-entry split
constexpr int JB_QSTACK = 64;              // query stacks: one entry per level at most (deeper trees flag ERR_STACK)
constexpr int JB_QT = 64;                  // query threads per block

struct JNode {
    uint32_t lo[3], size;
    uint32_t hi[3], pid;
    uint64_t pkey;
    uint32_t left, right;
    uint32_t ppt[3], pad;
};
struct JLeaf {
    uint32_t lo[3], cnt;
    uint32_t hi[3], sorted;
};
static_assert(sizeof(JNode) == 64, "node record");
static_assert(sizeof(JLeaf) == 32, "leaf record");

// device counters of an update
enum : uint32_t {
    C_NBUMP = 0, C_LBUMP, C_NTAKE, C_LTAKE, C_NCONS, C_LCONS, C_FLAGS, C_TASKS, C_RECS, C_BIG, C_ROOT, C_COUNT = 16
};
enum : uint32_t { F_OVERFLOW = 1u, F_BROKEN = 2u };

// A subtree the batch range [a, b) goes into; slot: where its result goes
// (record << 1 | side), or JB_NIL for the root.
struct JTask {
    uint32_t ref, a, b, slot;
};
// A join still to do: the pivot, the two sides (filled by the level below)
// and where the result goes; hit: a delete removed the pivot (Join2).
struct JRec {
    uint64_t kr;
    uint32_t left, right, slot, hit;
};
// A parallel BuildSorted over batch entries [a, a + n) (host-built table).
struct JBig {
    uint32_t a, n, slot, depth;
    uint64_t hoff;
};

struct Pools {
    JNode* node;
    JLeaf* leaf;
    uint64_t* lkey;
    uint32_t* lid;
    uint32_t* lpt;
    const uint32_t* nfree;
    const uint32_t* lfree;
    uint32_t nfree_n, lfree_n;
    uint32_t* ncons;
    uint32_t* lcons;
    uint32_t ncap, lcap, phi;
    uint32_t* ctr;
    // the update's batch in (key, id) order (points: insertions and builds)
    const uint64_t* bkey;
    const uint32_t* bid;
    const uint32_t* bpt;
    uint32_t bn;
    JRec* rec;
    uint32_t rcap;
};

// Entry references: a node's pivot (the node index), entry p of a leaf, or
// entry j of the batch.
constexpr uint64_t ER_LEAF = 1ull << 62, ER_BATCH = 2ull << 62, ER_KIND = 3ull << 62;
__device__ __forceinline__ uint64_t er_leaf(uint32_t l, uint32_t p) { return ER_LEAF | ((uint64_t)l << 8) | p; }
__device__ __forceinline__ uint64_t er_batch(uint32_t j) { return ER_BATCH | j; }

__device__ __forceinline__ void jb_broken(const Pools& P) { atomicOr(P.ctr + C_FLAGS, F_BROKEN); }
__device__ __forceinline__ void jb_overflow(const Pools& P) { atomicOr(P.ctr + C_FLAGS, F_OVERFLOW); }

__device__ __forceinline__ bool jb_like(uint64_t wa, uint64_t wb) {
    // alpha (wa + wb) <= min(wa, wb) with alpha = 1/5, in integers
    return wa + wb <= 5 * (wa < wb ? wa : wb);
}

__device__ void jb_key(const Pools& P, uint64_t r, uint64_t& key, uint32_t& id) {
    key = ~0ull;
    id = ~0u;
    const uint64_t kind = r & ER_KIND;
    if (kind == 0) {
        if (r >= P.ncap) return jb_broken(P);
        key = P.node[r].pkey;
        id = P.node[r].pid;
    } else if (kind == ER_LEAF) {
        const uint64_t l = (r & ~ER_KIND) >> 8, p = r & 255;
        if (l >= P.lcap || p >= P.phi) return jb_broken(P);
        key = P.lkey[l * P.phi + p];
        id = P.lid[l * P.phi + p];
    } else {
        const uint64_t j = r & ~ER_KIND;
        if (j >= P.bn) return jb_broken(P);
        key = P.bkey[j];
        id = P.bid[j];
    }
}

template <int D>
__device__ void jb_point(const Pools& P, uint64_t r, uint32_t* pt) {
#pragma unroll
    for (int d = 0; d < D; ++d) pt[d] = 0;
    const uint64_t kind = r & ER_KIND;
    if (kind == 0) {
        if (r >= P.ncap) return jb_broken(P);
#pragma unroll
        for (int d = 0; d < D; ++d) pt[d] = P.node[r].ppt[d];
    } else if (kind == ER_LEAF) {
        const uint64_t l = (r & ~ER_KIND) >> 8, p = r & 255;
        if (l >= P.lcap || p >= P.phi) return jb_broken(P);
#pragma unroll
        for (int d = 0; d < D; ++d) pt[d] = P.lpt[(l * P.phi + p) * D + d];
    } else {
        const uint64_t j = r & ~ER_KIND;
        if (j >= P.bn || !P.bpt) return jb_broken(P);
#pragma unroll
        for (int d = 0; d < D; ++d) pt[d] = P.bpt[j * D + d];
    }
}

__device__ __forceinline__ uint32_t jb_size(const Pools& P, uint32_t r) {
    if (r & JB_LEAF) {
        const uint32_t l = r & ~JB_LEAF;
        if (l >= P.lcap) {
            jb_broken(P);
            return 0;
        }
        return P.leaf[l].cnt;
    }
    if (r >= P.ncap) {
        jb_broken(P);
        return 0;
    }
    return P.node[r].size;
}

// Box of a subtree (lo = ~0, hi = 0 for an empty leaf).
template <int D>
__device__ void jb_box(const Pools& P, uint32_t r, uint32_t* lo, uint32_t* hi) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = 0xFFFFFFFFu;
        hi[d] = 0u;
    }
    if (r & JB_LEAF) {
        const uint32_t l = r & ~JB_LEAF;
        if (l >= P.lcap) return jb_broken(P);
        const JLeaf L = P.leaf[l];
        if (!L.cnt) return;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = L.lo[d];
            hi[d] = L.hi[d];
        }
        return;
    }
    if (r >= P.ncap) return jb_broken(P);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = P.node[r].lo[d];
        hi[d] = P.node[r].hi[d];
    }
}

// Allocation: the free lists of earlier updates first, then the bump
// pointer; a full pool flags an overflow (the update is run again).
__device__ uint32_t jb_alloc_node(const Pools& P) {
    const uint32_t t = atomicAdd(P.ctr + C_NTAKE, 1u);
    if (t < P.nfree_n) return P.nfree[P.nfree_n - 1 - t];
    const uint32_t b = atomicAdd(P.ctr + C_NBUMP, 1u);
    if (b >= P.ncap) {
        jb_overflow(P);
        return JB_NIL;
    }
    return b;
}
__device__ uint32_t jb_alloc_leaf(const Pools& P) {
    const uint32_t t = atomicAdd(P.ctr + C_LTAKE, 1u);
    if (t < P.lfree_n) return P.lfree[P.lfree_n - 1 - t];
    const uint32_t b = atomicAdd(P.ctr + C_LBUMP, 1u);
    if (b >= P.lcap) {
        jb_overflow(P);
        return JB_NIL;
    }
    return b;
}

// A node or leaf the new tree drops: freed after the commit.
__device__ void jb_consume(const Pools& P, uint32_t r) {
    if (r == JB_NIL) return;
    if (r & JB_LEAF) {
        const uint32_t l = r & ~JB_LEAF;
        if (l >= P.lcap) return jb_broken(P);
        const uint32_t i = atomicAdd(P.ctr + C_LCONS, 1u);
        if (i < P.lcap) P.lcons[i] = l;
        else jb_broken(P);
    } else {
        if (r >= P.ncap) return jb_broken(P);
        const uint32_t i = atomicAdd(P.ctr + C_NCONS, 1u);
        if (i < P.ncap) P.ncons[i] = r;
        else jb_broken(P);
    }
}

// A new leaf holding the entries seq[0 .. c) in that order.
template <int D>
__device__ uint32_t jb_new_leaf(const Pools& P, const uint64_t* seq, uint32_t c, uint32_t sorted) {
    const uint32_t l = jb_alloc_leaf(P);
    if (l == JB_NIL) return JB_NIL;
    if (c > P.phi) {
        jb_broken(P);
        c = P.phi;
    }
    uint32_t lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = 0xFFFFFFFFu;
        hi[d] = 0u;
    }
    const uint64_t base = (uint64_t)l * P.phi;
    for (uint32_t e = 0; e < c; ++e) {
        uint64_t k;
        uint32_t id, pt[D];
        jb_key(P, seq[e], k, id);
        jb_point<D>(P, seq[e], pt);
        P.lkey[base + e] = k;
        P.lid[base + e] = id;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            P.lpt[(base + e) * D + d] = pt[d];
            lo[d] = min(lo[d], pt[d]);
            hi[d] = max(hi[d], pt[d]);
        }
    }
    JLeaf L{};
#pragma unroll
    for (int d = 0; d < D; ++d) {
        L.lo[d] = lo[d];
        L.hi[d] = hi[d];
    }
    L.cnt = c;
    L.sorted = sorted;
    P.leaf[l] = L;
    return l | JB_LEAF;
}

// A new interior node (l, kr, r): box of both sides and the pivot.
template <int D>
__device__ uint32_t jb_new_node(const Pools& P, uint32_t l, uint64_t kr, uint32_t r) {
    const uint32_t v = jb_alloc_node(P);
    if (v == JB_NIL) return JB_NIL;
    uint32_t llo[D], lhi[D], rlo[D], rhi[D], pt[D];
    jb_box<D>(P, l, llo, lhi);
    jb_box<D>(P, r, rlo, rhi);
    jb_point<D>(P, kr, pt);
    JNode n{};
#pragma unroll
    for (int d = 0; d < D; ++d) {
        n.lo[d] = min(pt[d], min(llo[d], rlo[d]));
        n.hi[d] = max(pt[d], max(lhi[d], rhi[d]));
        n.ppt[d] = pt[d];
    }
    jb_key(P, kr, n.pkey, n.pid);
    n.size = jb_size(P, l) + 1 + jb_size(P, r);
    n.left = l;
    n.right = r;
    P.node[v] = n;
    return v;
}

// Entry references of leaf l in (key, id) order into out[0 .. count).
__device__ uint32_t jb_leaf_order(const Pools& P, uint32_t l, uint64_t* out) {
    if (l >= P.lcap) {
        jb_broken(P);
        return 0;
    }
    const JLeaf L = P.leaf[l];
    const uint32_t c = min(L.cnt, P.phi);
    const uint64_t base = (uint64_t)l * P.phi;
    if (L.sorted) {
        for (uint32_t e = 0; e < c; ++e) out[e] = er_leaf(l, e);
        return c;
    }
    for (uint32_t e = 0; e < c; ++e) {
        const uint64_t k = P.lkey[base + e];
        const uint32_t id = P.lid[base + e];
        uint32_t r = 0;
        for (uint32_t f = 0; f < c; ++f) r += pair_less(P.lkey[base + f], P.lid[base + f], k, id) ? 1u : 0u;
        if (r < c) out[r] = er_leaf(l, e);
        else jb_broken(P);
    }
    return c;
}

// Appends the entries of subtree t in (key, id) order to seq[c ..] (room
// up to cap) and drops every node and leaf of it. Only small subtrees
// (at most 2 phi entries) are flattened, so the walk is short.
__device__ void jb_collect(const Pools& P, uint32_t t, uint64_t* seq, uint32_t& c, uint32_t cap) {
    uint32_t stk[16];
    int sp = 0;
    uint32_t cur = t;
    for (int guard = 0; guard < 1024; ++guard) {
        while (!(cur & JB_LEAF)) {
            if (cur >= P.ncap || sp >= 16) return jb_broken(P);
            stk[sp++] = cur;
            cur = P.node[cur].left;
        }
        const uint32_t l = cur & ~JB_LEAF;
        if (l >= P.lcap) return jb_broken(P);
        if (c + P.leaf[l].cnt > cap) return jb_broken(P);
        c += jb_leaf_order(P, l, seq + c);
        jb_consume(P, cur);
        if (sp == 0) return;
        const uint32_t v = stk[--sp];
        if (c >= cap) return jb_broken(P);
        seq[c++] = v;  // the node's pivot
        jb_consume(P, v);
        cur = P.node[v].right;
    }
    jb_broken(P);
}

// Node(l, kr, r) keeping the leaf wrap: an interior node above 2 phi
// entries; two sorted leaves cut like BuildSorted's first step above phi;
// one leaf otherwise (two leaves are concatenated in their stored orders).
template <int D>
__device__ __noinline__ uint32_t jb_node(const Pools& P, uint32_t l, uint64_t kr, uint32_t r) {
    const uint32_t phi = P.phi;
    const uint32_t sl = jb_size(P, l), sr = jb_size(P, r);
    const uint32_t n = sl + 1 + sr;
    if (n > 2 * phi) return jb_new_node<D>(P, l, kr, r);
    constexpr uint32_t CAP = 2 * JB_PHI_MAX + 1;
    uint64_t seq[CAP];
    uint32_t c = 0;
    if (n <= phi && (l & JB_LEAF) && (r & JB_LEAF)) {
        const uint32_t li = l & ~JB_LEAF, ri = r & ~JB_LEAF;
        if (li >= P.lcap || ri >= P.lcap) {
            jb_broken(P);
            return JB_NIL;
        }
        for (uint32_t e = 0; e < sl; ++e) seq[c++] = er_leaf(li, e);
        seq[c++] = kr;
        for (uint32_t e = 0; e < sr; ++e) seq[c++] = er_leaf(ri, e);
        const uint32_t out = jb_new_leaf<D>(P, seq, c, P.leaf[li].sorted & P.leaf[ri].sorted);
        jb_consume(P, l);
        jb_consume(P, r);
        return out;
    }
    jb_collect(P, l, seq, c, CAP);
    if (c < CAP) seq[c++] = kr;
    jb_collect(P, r, seq, c, CAP);
    if (c != n) {
        jb_broken(P);
        return JB_NIL;
    }
    if (n <= phi) return jb_new_leaf<D>(P, seq, n, 1u);
    const uint32_t m = n / 2;
    const uint32_t a = jb_new_leaf<D>(P, seq, m, 1u);
    const uint32_t b = jb_new_leaf<D>(P, seq + m + 1, n - m - 1, 1u);
    return jb_new_node<D>(P, a, seq[m], b);
}

// Expose: (left, pivot, right) of an interior node, or of a non-empty leaf
// sorted and split like BuildSorted's first step. The node or leaf is dropped.
template <int D>
__device__ __noinline__ void jb_expose(const Pools& P, uint32_t t, uint32_t& l, uint64_t& kr, uint32_t& r) {
    l = r = JB_NIL;
    kr = 0;
    if (!(t & JB_LEAF)) {
        if (t >= P.ncap) return jb_broken(P);
        l = P.node[t].left;
        r = P.node[t].right;
        kr = t;
        jb_consume(P, t);
        return;
    }
    const uint32_t li = t & ~JB_LEAF;
    if (li >= P.lcap || P.leaf[li].cnt == 0) return jb_broken(P);
    uint64_t seq[JB_PHI_MAX];
    const uint32_t c = jb_leaf_order(P, li, seq);
    const uint32_t m = c / 2;
    l = jb_new_leaf<D>(P, seq, m, 1u);
    kr = seq[m];
    r = jb_new_leaf<D>(P, seq + m + 1, c - m - 1, 1u);
    jb_consume(P, t);
}

// Join(tl, kp, tr): Node() when the sides balance; otherwise down the
// heavier side's inner spine to the first subtree that balances with the
// other side, then back up with single or double rotations.
template <int D>
__device__ __noinline__ uint32_t jb_join(const Pools& P, uint32_t tl, uint64_t kp, uint32_t tr) {
    const uint64_t wl = jb_size(P, tl) + 1ull, wr = jb_size(P, tr) + 1ull;
    if (jb_like(wl, wr)) return jb_node<D>(P, tl, kp, tr);
    uint32_t sref[JB_STACK];
    uint64_t skey[JB_STACK];
    int sp = 0;
    if (wl > wr) {
        uint32_t cur = tl;
        while (!jb_like(jb_size(P, cur) + 1ull, wr)) {
            if (sp >= JB_STACK || cur == JB_NIL) {
                jb_broken(P);
                return JB_NIL;
            }
            uint32_t a, c;
            uint64_t k2;
            jb_expose<D>(P, cur, a, k2, c);
            sref[sp] = a;
            skey[sp] = k2;
            ++sp;
            cur = c;
        }
        uint32_t t2 = jb_node<D>(P, cur, kp, tr);
        while (sp > 0) {
            --sp;
            const uint32_t l = sref[sp];
            const uint64_t k2 = skey[sp];
            const uint64_t w = jb_size(P, l) + 1ull;
            if (jb_like(w, jb_size(P, t2) + 1ull)) {
                t2 = jb_node<D>(P, l, k2, t2);
                continue;
            }
            uint32_t l1, r1;
            uint64_t k3;
            jb_expose<D>(P, t2, l1, k3, r1);
            const uint64_t w1 = jb_size(P, l1) + 1ull, wr1 = jb_size(P, r1) + 1ull;
            if ((jb_like(w, w1) && jb_like(w + w1, wr1)) || w1 == 1) {  // single rotation
                const uint32_t x = jb_node<D>(P, l, k2, l1);
                t2 = jb_node<D>(P, x, k3, r1);
            } else {  // double rotation
                uint32_t a1, b1;
                uint64_t k4;
                jb_expose<D>(P, l1, a1, k4, b1);
                const uint32_t x = jb_node<D>(P, l, k2, a1);
                const uint32_t y = jb_node<D>(P, b1, k3, r1);
                t2 = jb_node<D>(P, x, k4, y);
            }
        }
        return t2;
    }
    uint32_t cur = tr;
    while (!jb_like(wl, jb_size(P, cur) + 1ull)) {
        if (sp >= JB_STACK || cur == JB_NIL) {
            jb_broken(P);
            return JB_NIL;
        }
        uint32_t c, b;
        uint64_t k2;
        jb_expose<D>(P, cur, c, k2, b);
        sref[sp] = b;
        skey[sp] = k2;
        ++sp;
        cur = c;
    }
    uint32_t t2 = jb_node<D>(P, tl, kp, cur);
    while (sp > 0) {
        --sp;
        const uint32_t r = sref[sp];
        const uint64_t k2 = skey[sp];
        const uint64_t w = jb_size(P, r) + 1ull;
        if (jb_like(jb_size(P, t2) + 1ull, w)) {
            t2 = jb_node<D>(P, t2, k2, r);
            continue;
        }
        uint32_t l1, r1;
        uint64_t k3;
        jb_expose<D>(P, t2, l1, k3, r1);
        const uint64_t wl1 = jb_size(P, l1) + 1ull, w1 = jb_size(P, r1) + 1ull;
        if ((jb_like(w1, w) && jb_like(w1 + w, wl1)) || w1 == 1) {  // single rotation
            const uint32_t y = jb_node<D>(P, r1, k2, r);
            t2 = jb_node<D>(P, l1, k3, y);
        } else {  // double rotation
            uint32_t a1, b1;
            uint64_t k4;
            jb_expose<D>(P, r1, a1, k4, b1);
            const uint32_t x = jb_node<D>(P, l1, k3, a1);
            const uint32_t y = jb_node<D>(P, b1, k2, r);
            t2 = jb_node<D>(P, x, k4, y);
        }
    }
    return t2;
}

// t without its largest entry, and that entry (t not empty).
template <int D>
__device__ __noinline__ uint32_t jb_split_last(const Pools& P, uint32_t t, uint64_t& kp) {
    uint32_t sref[JB_STACK];
    uint64_t skey[JB_STACK];
    int sp = 0;
    kp = 0;
    uint32_t cur = t;
    while (!(cur & JB_LEAF)) {
        if (cur >= P.ncap || sp >= JB_STACK) {
            jb_broken(P);
            return JB_NIL;
        }
        sref[sp] = P.node[cur].left;
        skey[sp] = cur;
        ++sp;
        jb_consume(P, cur);
        cur = P.node[cur].right;
    }
    const uint32_t li = cur & ~JB_LEAF;
    if (li >= P.lcap || P.leaf[li].cnt == 0) {
        jb_broken(P);
        return JB_NIL;
    }
    uint64_t seq[JB_PHI_MAX];
    const uint32_t c = jb_leaf_order(P, li, seq);
    kp = seq[c - 1];
    uint32_t r2 = jb_new_leaf<D>(P, seq, c - 1, 1u);
    jb_consume(P, cur);
    while (sp > 0) {
        --sp;
        r2 = jb_join<D>(P, sref[sp], skey[sp], r2);
    }
    return r2;
}

// Join2(l, r): the two sides of a deleted pivot joined with no middle entry.
template <int D>
__device__ uint32_t jb_join2(const Pools& P, uint32_t l, uint32_t r) {
    if (jb_size(P, l) == 0) {
        jb_consume(P, l);
        return r;
    }
    uint64_t kp;
    const uint32_t l2 = jb_split_last<D>(P, l, kp);
    return jb_join<D>(P, l2, kp, r);
}

// BuildSorted over seq[0 .. n) with n < 4 phi (two levels of interior
// nodes at most).
template <int D>
__device__ uint32_t jb_build_small(const Pools& P, const uint64_t* seq, uint32_t n) {
    const uint32_t phi = P.phi;
    if (n <= phi) return jb_new_leaf<D>(P, seq, n, 1u);
    uint32_t side[2];
    const uint32_t m = n / 2;
    const uint64_t* s[2] = {seq, seq + m + 1};
    const uint32_t k[2] = {m, n - m - 1};
    for (int x = 0; x < 2; ++x) {
        if (k[x] <= phi) {
            side[x] = jb_new_leaf<D>(P, s[x], k[x], 1u);
            continue;
        }
        const uint32_t h = k[x] / 2;
        if (h > phi || k[x] - h - 1 > phi) {
            jb_broken(P);
            side[x] = JB_NIL;
            continue;
        }
        const uint32_t a = jb_new_leaf<D>(P, s[x], h, 1u);
        const uint32_t b = jb_new_leaf<D>(P, s[x] + h + 1, k[x] - h - 1, 1u);
        side[x] = jb_new_node<D>(P, a, s[x][h], b);
    }
    return jb_new_node<D>(P, side[0], seq[m], side[1]);
}

__device__ void jb_deliver(const Pools& P, uint32_t slot, uint32_t ref) {
    if (slot == JB_NIL) {
        P.ctr[C_ROOT] = ref;
        return;
    }
    const uint32_t r = slot >> 1;
    if (r >= P.rcap) return jb_broken(P);
    if (slot & 1) P.rec[r].right = ref;
    else P.rec[r].left = ref;
}

__device__ uint32_t jb_new_rec(const Pools& P, uint64_t kr, uint32_t slot, uint32_t hit) {
    const uint32_t r = atomicAdd(P.ctr + C_RECS, 1u);
    if (r >= P.rcap) {
        jb_overflow(P);
        return JB_NIL;
    }
    JRec x;
    x.kr = kr;
    x.left = x.right = JB_NIL;
    x.slot = slot;
    x.hit = hit;
    P.rec[r] = x;
    return r;
}

__device__ void jb_push(const Pools& P, JTask* out, uint32_t cap, uint32_t* ctr, uint32_t ref, uint32_t a,
                        uint32_t b, uint32_t slot) {
    const uint32_t i = atomicAdd(ctr, 1u);
    if (i >= cap) return jb_overflow(P);
    out[i] = JTask{ref, a, b, slot};
}

// First batch entry in [a, b) not below (key, id).
__device__ uint32_t jb_lower(const Pools& P, uint32_t a, uint32_t b, uint64_t key, uint32_t id) {
    while (a < b) {
        const uint32_t m = a + (b - a) / 2;
        if (pair_less(P.bkey[m], P.bid[m], key, id)) a = m + 1;
        else b = m;
    }
    return a;
}

// Sends the batch ranges [a, c) and [c2, b) of record r to its two sides:
// an empty range leaves that side as it is.
__device__ void jb_split(const Pools& P, uint32_t r, uint32_t lref, uint32_t rref, uint32_t a, uint32_t c,
                         uint32_t c2, uint32_t b, JTask* tout, uint32_t tcap) {
    if (c == a) P.rec[r].left = lref;
    else jb_push(P, tout, tcap, P.ctr + C_TASKS, lref, a, c, r << 1);
    if (c2 >= b) P.rec[r].right = rref;
    else jb_push(P, tout, tcap, P.ctr + C_TASKS, rref, c2, b, (r << 1) | 1u);
}

// Batch insertion, one level down (Alg. 4).
template <int D>
__global__ __launch_bounds__(64) void k_jb_ins_down(Pools P, const JTask* __restrict__ tin, uint32_t nt,
                                                    JTask* __restrict__ tout, uint32_t tcap, JTask* __restrict__ big,
                                                    uint32_t bcap) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += gridDim.x * blockDim.x) {
        const JTask T = tin[i];
        if (T.b > P.bn || T.a > T.b) {
            jb_broken(P);
            continue;
        }
        if (T.a == T.b) {
            jb_deliver(P, T.slot, T.ref);
            continue;
        }
        const uint32_t phi = P.phi, n = T.b - T.a;
        if (!(T.ref & JB_LEAF)) {
            if (T.ref >= P.ncap) {
                jb_broken(P);
                continue;
            }
            const JNode N = P.node[T.ref];
            const uint32_t c = jb_lower(P, T.a, T.b, N.pkey, N.pid);
            const uint32_t r = jb_new_rec(P, T.ref, T.slot, 0u);
            if (r == JB_NIL) continue;
            jb_consume(P, T.ref);
            jb_split(P, r, N.left, N.right, T.a, c, c, T.b, tout, tcap);
            continue;
        }
        const uint32_t li = T.ref & ~JB_LEAF;
        if (li >= P.lcap) {
            jb_broken(P);
            continue;
        }
        const uint32_t m = P.leaf[li].cnt;
        if (m + n <= phi) {  // appended, order relaxed
            uint64_t seq[JB_PHI_MAX];
            uint32_t c = 0;
            for (uint32_t e = 0; e < m; ++e) seq[c++] = er_leaf(li, e);
            for (uint32_t j = T.a; j < T.b; ++j) seq[c++] = er_batch(j);
            jb_deliver(P, T.slot, jb_new_leaf<D>(P, seq, c, m == 0 ? 1u : 0u));
            jb_consume(P, T.ref);
        } else if (m + n < 4 * phi) {  // local rebuild
            uint64_t ls[JB_PHI_MAX];
            const uint32_t lc = jb_leaf_order(P, li, ls);
            uint64_t seq[4 * JB_PHI_MAX];
            uint32_t c = 0, x = 0, j = T.a;
            while ((x < lc || j < T.b) && c < 4 * JB_PHI_MAX) {
                bool from_leaf = j >= T.b;
                if (x < lc && j < T.b) {
                    uint64_t k;
                    uint32_t id;
                    jb_key(P, ls[x], k, id);
                    from_leaf = pair_less(k, id, P.bkey[j], P.bid[j]);
                }
                seq[c++] = from_leaf ? ls[x++] : er_batch(j++);
            }
            jb_deliver(P, T.slot, jb_build_small<D>(P, seq, c));
            jb_consume(P, T.ref);
        } else if (m == 0) {  // an empty leaf and a large share: parallel BuildSorted
            jb_push(P, big, bcap, P.ctr + C_BIG, JB_NIL, T.a, T.b, T.slot);
            jb_consume(P, T.ref);
        } else {  // exposed, then on down
            uint32_t l, r;
            uint64_t kr;
            jb_expose<D>(P, T.ref, l, kr, r);
            uint64_t key;
            uint32_t id;
            jb_key(P, kr, key, id);
            const uint32_t c = jb_lower(P, T.a, T.b, key, id);
            const uint32_t rr = jb_new_rec(P, kr, T.slot, 0u);
            if (rr == JB_NIL) continue;
            jb_split(P, rr, l, r, T.a, c, c, T.b, tout, tcap);
        }
    }
}

// Batch deletion, one level down: the batch holds the (key, id) pairs of
// live entries; an interior node whose pivot is among them is joined by Join2.
template <int D>
__global__ __launch_bounds__(64) void k_jb_del_down(Pools P, const JTask* __restrict__ tin, uint32_t nt,
                                                    JTask* __restrict__ tout, uint32_t tcap) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += gridDim.x * blockDim.x) {
        const JTask T = tin[i];
        if (T.b > P.bn || T.a > T.b) {
            jb_broken(P);
            continue;
        }
        if (T.a == T.b) {
            jb_deliver(P, T.slot, T.ref);
            continue;
        }
        if (!(T.ref & JB_LEAF)) {
            if (T.ref >= P.ncap) {
                jb_broken(P);
                continue;
            }
            const JNode N = P.node[T.ref];
            const uint32_t c = jb_lower(P, T.a, T.b, N.pkey, N.pid);
            const uint32_t hit = c < T.b && P.bkey[c] == N.pkey && P.bid[c] == N.pid;
            const uint32_t r = jb_new_rec(P, T.ref, T.slot, hit);
            if (r == JB_NIL) continue;
            jb_consume(P, T.ref);
            jb_split(P, r, N.left, N.right, T.a, c, c + hit, T.b, tout, tcap);
            continue;
        }
        const uint32_t li = T.ref & ~JB_LEAF;
        if (li >= P.lcap) {
            jb_broken(P);
            continue;
        }
        const JLeaf L = P.leaf[li];
        const uint64_t base = (uint64_t)li * P.phi;
        uint64_t seq[JB_PHI_MAX];
        uint32_t c = 0;
        for (uint32_t e = 0; e < L.cnt && e < P.phi; ++e) {
            const uint64_t k = P.lkey[base + e];
            const uint32_t id = P.lid[base + e];
            const uint32_t p = jb_lower(P, T.a, T.b, k, id);
            if (!(p < T.b && P.bkey[p] == k && P.bid[p] == id)) seq[c++] = er_leaf(li, e);
        }
        if (c == L.cnt) {
            jb_deliver(P, T.slot, T.ref);
            continue;
        }
        jb_deliver(P, T.slot, jb_new_leaf<D>(P, seq, c, L.sorted));
        jb_consume(P, T.ref);
    }
}

// One level up: every record joins its two sides.
template <int D>
__global__ __launch_bounds__(64) void k_jb_up(Pools P, uint32_t r0, uint32_t r1) {
    for (uint32_t i = r0 + blockIdx.x * blockDim.x + threadIdx.x; i < r1; i += gridDim.x * blockDim.x) {
        if (i >= P.rcap) {
            jb_broken(P);
            continue;
        }
        const JRec R = P.rec[i];
        if (R.left == JB_NIL || R.right == JB_NIL) {
            jb_broken(P);
            continue;
        }
        const uint32_t res = R.hit ? jb_join2<D>(P, R.left, R.right) : jb_join<D>(P, R.left, R.kr, R.right);
        jb_deliver(P, R.slot, res);
    }
}

// ---------------------------------------------- parallel BuildSorted
// Sorted range of heap position v of BuildSorted over n entries, or false
// when an ancestor is already a leaf (the position is not in the shape).
__device__ __forceinline__ bool jb_heap_range(uint64_t v, uint32_t n, uint32_t phi, uint32_t& a, uint32_t& b) {
    const uint64_t x = v + 1;
    const int d = 63 - __builtin_clzll(x);
    a = 0;
    b = n;
    for (int s = d - 1; s >= 0; --s) {
        if (b - a <= phi) return false;
        const uint32_t m = a + (b - a) / 2;
        if ((x >> s) & 1u) a = m + 1;
        else b = m;
    }
    return true;
}

__device__ __forceinline__ uint32_t jb_big_of(const JBig* bt, uint32_t nbt, uint64_t g) {
    uint32_t lo = 0, hi = nbt;  // last task with hoff <= g
    while (hi - lo > 1) {
        const uint32_t m = (lo + hi) / 2;
        if (bt[m].hoff <= g) lo = m;
        else hi = m;
    }
    return lo;
}

__global__ void k_jb_bb_flags(const JBig* __restrict__ bt, uint32_t nbt, uint64_t HT, uint32_t phi,
                              uint32_t* __restrict__ isl, uint32_t* __restrict__ isn) {
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < HT; g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t t = jb_big_of(bt, nbt, g);
        uint32_t a, b;
        const bool ex = jb_heap_range(g - bt[t].hoff, bt[t].n, phi, a, b);
        isl[g] = ex && b - a <= phi;
        isn[g] = ex && b - a > phi;
    }
}

__device__ __forceinline__ uint32_t jb_heap_ref(uint64_t g, const uint32_t* isl, const uint32_t* offl,
                                                const uint32_t* offn, uint32_t lbase, uint32_t nbase) {
    return isl[g] ? ((lbase + offl[g]) | JB_LEAF) : (nbase + offn[g]);
}

template <int D>
__global__ void k_jb_bb_write(Pools P, const JBig* __restrict__ bt, uint32_t nbt, uint64_t HT,
                              const uint32_t* __restrict__ isl, const uint32_t* __restrict__ isn,
                              const uint32_t* __restrict__ offl, const uint32_t* __restrict__ offn, uint32_t lbase,
                              uint32_t nbase) {
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < HT; g += (uint64_t)gridDim.x * blockDim.x) {
        if (!isl[g] && !isn[g]) continue;
        const uint32_t t = jb_big_of(bt, nbt, g);
        const uint64_t v = g - bt[t].hoff;
        uint32_t ra, rb;
        jb_heap_range(v, bt[t].n, P.phi, ra, rb);
        const uint32_t a0 = bt[t].a;
        uint32_t ref;
        if (isl[g]) {
            const uint32_t l = lbase + offl[g];
            if (l >= P.lcap || rb - ra > P.phi || (uint64_t)a0 + rb > P.bn) {
                jb_broken(P);
                continue;
            }
            const uint64_t base = (uint64_t)l * P.phi;
            JLeaf L{};
#pragma unroll
            for (int d = 0; d < D; ++d) {
                L.lo[d] = 0xFFFFFFFFu;
                L.hi[d] = 0u;
            }
            for (uint32_t e = 0; e < rb - ra; ++e) {
                const uint64_t j = (uint64_t)a0 + ra + e;
                P.lkey[base + e] = P.bkey[j];
                P.lid[base + e] = P.bid[j];
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const uint32_t p = P.bpt[j * D + d];
                    P.lpt[(base + e) * D + d] = p;
                    L.lo[d] = min(L.lo[d], p);
                    L.hi[d] = max(L.hi[d], p);
                }
            }
            L.cnt = rb - ra;
            L.sorted = 1;
            P.leaf[l] = L;
            ref = l | JB_LEAF;
        } else {
            const uint32_t vi = nbase + offn[g];
            const uint64_t g0 = bt[t].hoff + 2 * v + 1;
            const uint64_t j = (uint64_t)a0 + ra + (rb - ra) / 2;
            if (vi >= P.ncap || g0 + 1 >= HT || j >= P.bn) {
                jb_broken(P);
                continue;
            }
            JNode N{};
            N.pkey = P.bkey[j];
            N.pid = P.bid[j];
#pragma unroll
            for (int d = 0; d < D; ++d) N.ppt[d] = P.bpt[j * D + d];
            N.size = rb - ra;
            N.left = jb_heap_ref(g0, isl, offl, offn, lbase, nbase);
            N.right = jb_heap_ref(g0 + 1, isl, offl, offn, lbase, nbase);
            P.node[vi] = N;  // its box: k_jb_bb_box
            ref = vi;
        }
        if (v == 0) jb_deliver(P, bt[t].slot, ref);
    }
}

// Boxes of the interior nodes at heap depth d (their children are done).
template <int D>
__global__ void k_jb_bb_box(Pools P, const JBig* __restrict__ bt, uint32_t nbt, uint64_t HT,
                            const uint32_t* __restrict__ isn, const uint32_t* __restrict__ offn, uint32_t nbase,
                            uint32_t d) {
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < HT; g += (uint64_t)gridDim.x * blockDim.x) {
        if (!isn[g]) continue;
        const uint32_t t = jb_big_of(bt, nbt, g);
        const uint64_t v = g - bt[t].hoff;
        if ((uint32_t)(63 - __builtin_clzll(v + 1)) != d) continue;
        const uint32_t vi = nbase + offn[g];
        if (vi >= P.ncap) {
            jb_broken(P);
            continue;
        }
        JNode N = P.node[vi];
        uint32_t llo[D], lhi[D], rlo[D], rhi[D];
        jb_box<D>(P, N.left, llo, lhi);
        jb_box<D>(P, N.right, rlo, rhi);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            N.lo[k] = min(N.ppt[k], min(llo[k], rlo[k]));
            N.hi[k] = max(N.ppt[k], max(lhi[k], rhi[k]));
        }
        P.node[vi] = N;
    }
}

// Commit: the entries the update took off the free lists are gone; the
// nodes and leaves it dropped go on them.
__global__ void k_jb_commit(uint32_t* __restrict__ nfree, uint32_t nbase, const uint32_t* __restrict__ ncons,
                            uint32_t nc, uint32_t* __restrict__ lfree, uint32_t lbase,
                            const uint32_t* __restrict__ lcons, uint32_t lc) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nc; j += stride) nfree[nbase + j] = ncons[j];
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < lc; j += stride) lfree[lbase + j] = lcons[j];
}

// ------------------------------------------------------------- deletes
// Claims the live ids among ids[0 .. m) (alive word 1 -> 0) and lists
// their (key, id) pairs.
__global__ void k_jb_claim(const uint32_t* __restrict__ ids, uint64_t m, uint32_t next_id, uint32_t* __restrict__ alive,
                           const uint64_t* __restrict__ idkey, uint64_t* __restrict__ dk, uint32_t* __restrict__ di,
                           unsigned long long* __restrict__ nd) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t id = ids[j];
        if (id < next_id && atomicExch(alive + id, 0u) == 1u) {
            const unsigned long long p = atomicAdd(nd, 1ull);
            dk[p] = idkey[id];
            di[p] = id;
        }
    }
}

template <int D>
__global__ void k_jb_gather(const uint32_t* __restrict__ ids, uint64_t n, const uint32_t* __restrict__ src,
                            uint32_t id_base, uint32_t* __restrict__ out) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t j = ids[i] - id_base;
#pragma unroll
        for (int d = 0; d < D; ++d) out[i * D + d] = src[j * D + d];
    }
}

__global__ void k_jb_fill(uint32_t* __restrict__ p, uint64_t a, uint64_t b, uint32_t v) {
    for (uint64_t i = a + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_jb_copy_u64(uint64_t* __restrict__ dst, const uint64_t* __restrict__ src, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_jb_iota(uint32_t* __restrict__ p, uint64_t m, uint32_t base) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = base + (uint32_t)i;
}

// ------------------------------------------------------------- queries
// The read-only view queries take.
struct JView {
    const JNode* node;
    const JLeaf* leaf;
    const uint32_t* lid;
    const uint32_t* lpt;
    uint32_t ncap, lcap, phi, root;
};

template <int D>
__device__ __forceinline__ bool jv_box(const JView& t, uint32_t r, uint32_t* lo, uint32_t* hi) {
    if (r & JB_LEAF) {
        const uint32_t l = r & ~JB_LEAF;
        if (l >= t.lcap) return false;
        const JLeaf L = t.leaf[l];
        if (!L.cnt) return false;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = L.lo[d];
            hi[d] = L.hi[d];
        }
        return true;
    }
    if (r >= t.ncap) return false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = t.node[r].lo[d];
        hi[d] = t.node[r].hi[d];
    }
    return true;
}

template <int D>
__device__ __forceinline__ uint64_t jv_dist(const JView& t, const uint32_t* q, uint32_t r) {
    uint32_t lo[D], hi[D];
    if (!jv_box<D>(t, r, lo, hi)) return PAD_D2;
    uint64_t s = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const uint32_t x = q[d] < lo[d] ? lo[d] - q[d] : (q[d] > hi[d] ? q[d] - hi[d] : 0u);
        s += (uint64_t)x * x;
    }
    return s;
}

// kNN, a thread per query (k <= 16): depth first, nearer child first,
// pruning boxes farther than the k-th distance; every interior node's
// pivot is a candidate, leaves are scanned. The stack of pending subtrees
// is in LDS.
template <int D, int K>
__global__ __launch_bounds__(JB_QT) void k_jb_knn(JView t, const uint32_t* __restrict__ qp, uint64_t nq,
                                                  const uint32_t* __restrict__ order, uint32_t* __restrict__ out_ids,
                                                  uint64_t* __restrict__ out_d2, uint32_t* __restrict__ err) {
    __shared__ uint32_t s_stk[JB_QSTACK][JB_QT];
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
    auto take = [&](const uint32_t* p, uint32_t id) {
        const uint64_t dd = pt_dist<D>(q, p);
        if (pair_less(dd, id, bd[K - 1], bi[K - 1])) topk_insert<K>(bd, bi, dd, id);
    };
    // depth first: the nearer child next, the farther one on the stack (its
    // box distance tested again when it is taken off)
    uint32_t* stk = &s_stk[0][threadIdx.x];
    int sp = 0;
    uint32_t v = t.root;
    uint64_t dv = v != JB_NIL ? jv_dist<D>(t, q, v) : PAD_D2;
    for (uint32_t guard = 0;; ++guard) {
        if (guard >= (1u << 26)) {  // more steps than any tree of 2^31 points takes
            atomicOr(err, ERR_STACK);
            break;
        }
        bool next = false;
        if (v != JB_NIL && dv <= bd[K - 1]) {
            if (v & JB_LEAF) {
                const uint32_t l = v & ~JB_LEAF;
                if (l < t.lcap) {
                    const uint32_t c = min(t.leaf[l].cnt, t.phi);
                    const uint64_t base = (uint64_t)l * t.phi;
                    for (uint32_t e = 0; e < c; ++e) take(t.lpt + (base + e) * D, t.lid[base + e]);
                }
            } else if (v < t.ncap) {
                const JNode N = t.node[v];
                take(N.ppt, N.pid);
                const uint64_t d0 = jv_dist<D>(t, q, N.left), d1 = jv_dist<D>(t, q, N.right);
                const uint32_t fa = d0 <= d1 ? N.right : N.left, ne = d0 <= d1 ? N.left : N.right;
                const uint64_t dfa = d0 <= d1 ? d1 : d0, dne = d0 <= d1 ? d0 : d1;
                if (dfa <= bd[K - 1]) {
                    if (sp >= JB_QSTACK) {
                        atomicOr(err, ERR_STACK);
                        break;
                    }
                    stk[(sp++) * JB_QT] = fa;
                }
                v = ne;
                dv = dne;
                next = true;
            }
        }
        if (next) continue;
        if (sp == 0) break;
        v = stk[(--sp) * JB_QT];
        dv = jv_dist<D>(t, q, v);
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        out_ids[qi * K + j] = bi[j];
        out_d2[qi * K + j] = bd[j];
    }
}

// Range count (REPORT = false) or report, a thread per box. A subtree
// inside the box counts its size, or has all its entries reported; a
// straddling leaf is scanned; a straddling interior node tests its pivot.
template <int D, bool REPORT>
__global__ __launch_bounds__(JB_QT) void k_jb_range(JView t, const uint32_t* __restrict__ boxes, uint64_t nb,
                                                    const uint32_t* __restrict__ order, uint64_t* __restrict__ counts,
                                                    const uint64_t* __restrict__ offsets, uint32_t* __restrict__ out,
                                                    uint32_t* __restrict__ err) {
    __shared__ uint32_t s_stk[JB_QSTACK][JB_QT];
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
    auto in_box = [&](const uint32_t* p) {
        bool in = true;
#pragma unroll
        for (int d = 0; d < D; ++d) in = in && lo[d] <= p[d] && p[d] <= hi[d];
        return in;
    };
    auto emit = [&](uint32_t id) {
        if (!REPORT) ++cnt;
        else if (o < lim) out[o++] = id;
    };
    uint32_t* stk = &s_stk[0][threadIdx.x];
    int sp = 0;
    if (!empty && t.root != JB_NIL) stk[(sp++) * JB_QT] = t.root;
    for (uint32_t guard = 0; sp > 0; ++guard) {
        if (guard >= (1u << 28)) {  // more steps than a walk over every node of 2^31 points takes
            atomicOr(err, ERR_STACK);
            break;
        }
        const uint32_t w = stk[(--sp) * JB_QT];
        const bool known = (w & JB_IN) != 0;
        const uint32_t v = w & ~JB_IN;
        bool inside = known;
        if (!known) {
            uint32_t blo[D], bhi[D];
            if (!jv_box<D>(t, v, blo, bhi)) continue;
            bool meets = true;
            inside = true;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                meets = meets && !(bhi[d] < lo[d] || blo[d] > hi[d]);
                inside = inside && lo[d] <= blo[d] && bhi[d] <= hi[d];
            }
            if (!meets) continue;
        }
        if (v & JB_LEAF) {
            const uint32_t l = v & ~JB_LEAF;
            if (l >= t.lcap) continue;
            const uint32_t c = min(t.leaf[l].cnt, t.phi);
            if (inside && !REPORT) {
                cnt += c;
                continue;
            }
            const uint64_t base = (uint64_t)l * t.phi;
            for (uint32_t e = 0; e < c; ++e)
                if (inside || in_box(t.lpt + (base + e) * D)) emit(t.lid[base + e]);
            continue;
        }
        if (v >= t.ncap) continue;
        const JNode N = t.node[v];
        if (inside && !REPORT) {
            cnt += N.size;
            continue;
        }
        if (inside || in_box(N.ppt)) emit(N.pid);
        if (sp + 2 > JB_QSTACK) {
            atomicOr(err, ERR_STACK);
            break;
        }
        const uint32_t f = inside ? JB_IN : 0u;
        stk[(sp++) * JB_QT] = N.right | f;
        stk[(sp++) * JB_QT] = N.left | f;
    }
    if (!REPORT) counts[b] = cnt;
}

}  // namespace
}  // namespace psi

using namespace psi;

struct psi_bst_s {
    psi_index ix = nullptr;  // stream, encode and sort workspace, query ordering, error word
    uint32_t D = 3, curve = 1, phi = 40;
    uint64_t n = 0;
    uint32_t next_id = 0;
    uint32_t root = JB_NIL;
    // pools: capacities, bump pointers, free-list lengths
    uint32_t ncap = 0, lcap = 0, nbump = 0, lbump = 0, nfree_n = 0, lfree_n = 0;
    Buf node, leaf, lkey, lid, lpt, nfree, lfree, ncons, lcons;
    // update workspace
    Buf ctr, task[2], rec, big, bigtab, isl, isn, offl, offn, tot, tmp;
    Buf alive, idkey, kin, bpts, dk, di, nd;
};

namespace {

uint32_t jb_depth(uint64_t n, uint32_t phi) {
    uint32_t d = 0;
    for (uint64_t s = n; s > phi; s /= 2) ++d;
    return d;
}

// Pools of at least nn nodes and nl leaves (contents kept).
psi_status jb_grow(psi_bst t, uint64_t nn, uint64_t nl) {
    hipStream_t st = t->ix->st;
    psi_status s;
    nn = std::max<uint64_t>(nn, 16);
    nl = std::max<uint64_t>(nl, 16);
    if (nn > (1u << 30) || nl > (1u << 30)) return PSI_E_CAPACITY;
    const uint64_t phi = t->phi;
    if (nn > t->ncap) {
        const uint64_t keep = t->ncap;
        if ((s = t->node.grow_keep(nn * sizeof(JNode), keep * sizeof(JNode), st)) != PSI_OK) return s;
        if ((s = t->nfree.grow_keep(nn * 4, keep * 4, st)) != PSI_OK) return s;
        if ((s = t->ncons.grow_keep(nn * 4, keep * 4, st)) != PSI_OK) return s;  // a growth mid-update keeps the list
        t->ncap = (uint32_t)std::min<uint64_t>({t->node.bytes / sizeof(JNode), t->nfree.bytes / 4, t->ncons.bytes / 4,
                                                 1ull << 30});
    }
    if (nl > t->lcap) {
        const uint64_t keep = t->lcap;
        if ((s = t->leaf.grow_keep(nl * sizeof(JLeaf), keep * sizeof(JLeaf), st)) != PSI_OK) return s;
        if ((s = t->lkey.grow_keep(nl * phi * 8, keep * phi * 8, st)) != PSI_OK) return s;
        if ((s = t->lid.grow_keep(nl * phi * 4, keep * phi * 4, st)) != PSI_OK) return s;
        if ((s = t->lpt.grow_keep(nl * phi * 4 * t->D, keep * phi * 4 * t->D, st)) != PSI_OK) return s;
        if ((s = t->lfree.grow_keep(nl * 4, keep * 4, st)) != PSI_OK) return s;
        if ((s = t->lcons.grow_keep(nl * 4, keep * 4, st)) != PSI_OK) return s;
        t->lcap = (uint32_t)std::min<uint64_t>({t->leaf.bytes / sizeof(JLeaf), t->lkey.bytes / (phi * 8),
                                                 t->lid.bytes / (phi * 4), t->lpt.bytes / (phi * 4 * t->D),
                                                 t->lfree.bytes / 4, t->lcons.bytes / 4, 1ull << 30});
    }
    return PSI_OK;
}

Pools jb_pools(psi_bst t, const uint64_t* bk, const uint32_t* bi, const uint32_t* bp, uint32_t bn) {
    Pools P{};
    P.node = t->node.as<JNode>();
    P.leaf = t->leaf.as<JLeaf>();
    P.lkey = t->lkey.as<uint64_t>();
    P.lid = t->lid.as<uint32_t>();
    P.lpt = t->lpt.as<uint32_t>();
    P.nfree = t->nfree.as<uint32_t>();
    P.lfree = t->lfree.as<uint32_t>();
    P.nfree_n = t->nfree_n;
    P.lfree_n = t->lfree_n;
    P.ncons = t->ncons.as<uint32_t>();
    P.lcons = t->lcons.as<uint32_t>();
    P.ncap = t->ncap;
    P.lcap = t->lcap;
    P.phi = t->phi;
    P.ctr = t->ctr.as<uint32_t>();
    P.bkey = bk;
    P.bid = bi;
    P.bpt = bp;
    P.bn = bn;
    P.rec = t->rec.as<JRec>();
    P.rcap = (uint32_t)std::min<uint64_t>(t->rec.bytes / sizeof(JRec), 1u << 30);
    return P;
}

JView jb_view(psi_bst t) {
    JView v{};
    v.node = t->node.as<JNode>();
    v.leaf = t->leaf.as<JLeaf>();
    v.lid = t->lid.as<uint32_t>();
    v.lpt = t->lpt.as<uint32_t>();
    v.ncap = t->ncap;
    v.lcap = t->lcap;
    v.phi = t->phi;
    v.root = t->root;
    return v;
}

// The device counters, read back (waits for the stream).
psi_status jb_counters(psi_bst t, uint32_t* h) {
    psi_status s = readback(t->ix, t->ctr.p, C_COUNT * 4);
    if (s == PSI_OK) std::memcpy(h, t->ix->pinned, C_COUNT * 4);
    return s;
}

psi_status jb_set_counters(psi_bst t, const uint32_t* h) {
    std::memcpy(t->ix->pinned, h, C_COUNT * 4);
    psi_status s = hip_ok(hipMemcpyAsync(t->ctr.p, t->ix->pinned, C_COUNT * 4, hipMemcpyHostToDevice, t->ix->st));
    if (s == PSI_OK) s = hip_ok(hipStreamSynchronize(t->ix->st));
    return s;
}

// Parallel BuildSorted of the tasks' batch ranges; each result goes to its
// slot. Allocates from the bump pointers (growing the pools if needed).
psi_status jb_big_builds(psi_bst t, const std::vector<JTask>& tasks, const uint64_t* bk, const uint32_t* bi,
                         const uint32_t* bp, uint32_t bn, uint32_t* h_ctr) {
    hipStream_t st = t->ix->st;
    psi_status s;
    std::vector<JBig> tab(tasks.size());
    uint64_t HT = 0;
    uint32_t maxd = 0;
    for (size_t i = 0; i < tasks.size(); ++i) {
        if (tasks[i].b < tasks[i].a || tasks[i].b > bn) return PSI_E_INTERNAL;
        tab[i].a = tasks[i].a;
        tab[i].n = tasks[i].b - tasks[i].a;
        tab[i].slot = tasks[i].slot;
        tab[i].depth = jb_depth(tab[i].n, t->phi);
        tab[i].hoff = HT;
        HT += (2ull << tab[i].depth) - 1;
        maxd = std::max(maxd, tab[i].depth);
    }
    if (HT >= (1ull << 32)) return PSI_E_CAPACITY;
    if ((s = t->bigtab.ensure(tab.size() * sizeof(JBig))) != PSI_OK) return s;
    for (Buf* b : {&t->isl, &t->isn, &t->offl, &t->offn})
        if ((s = b->ensure((HT + 1) * 4)) != PSI_OK) return s;
    if ((s = t->tot.ensure(16)) != PSI_OK) return s;
    if ((s = t->tmp.ensure((scan_tmp_words(HT) + 8) * 4)) != PSI_OK) return s;
    if ((s = hip_ok(hipMemcpy(t->bigtab.p, tab.data(), tab.size() * sizeof(JBig), hipMemcpyHostToDevice))) != PSI_OK)
        return s;
    const uint32_t nbt = (uint32_t)tab.size();
    const JBig* bt = t->bigtab.as<JBig>();
    hipLaunchKernelGGL(k_jb_bb_flags, dim3(blocks_of(HT, 256)), dim3(256), 0, st, bt, nbt, HT, t->phi,
                       t->isl.as<uint32_t>(), t->isn.as<uint32_t>());
    launch_scan_u32(st, t->isl.as<uint32_t>(), t->offl.as<uint32_t>(), HT, t->tot.as<uint32_t>(), t->tmp.as<uint32_t>());
    launch_scan_u32(st, t->isn.as<uint32_t>(), t->offn.as<uint32_t>(), HT, t->tot.as<uint32_t>() + 1,
                    t->tmp.as<uint32_t>());
    if ((s = readback(t->ix, t->tot.p, 8)) != PSI_OK) return s;
    uint32_t tot[2];
    std::memcpy(tot, t->ix->pinned, 8);
    const uint32_t lbase = h_ctr[C_LBUMP], nbase = h_ctr[C_NBUMP];
    if ((s = jb_grow(t, (uint64_t)nbase + tot[1], (uint64_t)lbase + tot[0])) != PSI_OK) return s;
    h_ctr[C_LBUMP] = lbase + tot[0];
    h_ctr[C_NBUMP] = nbase + tot[1];
    if ((s = jb_set_counters(t, h_ctr)) != PSI_OK) return s;
    const Pools P = jb_pools(t, bk, bi, bp, bn);
    const unsigned g = blocks_of(HT, 256);
#define PSI_JBW(DD)                                                                                                \
    hipLaunchKernelGGL(k_jb_bb_write<DD>, dim3(g), dim3(256), 0, st, P, bt, nbt, HT, t->isl.as<uint32_t>(),         \
                       t->isn.as<uint32_t>(), t->offl.as<uint32_t>(), t->offn.as<uint32_t>(), lbase, nbase);       \
    for (int d = (int)maxd - 1; d >= 0; --d)                                                                        \
        hipLaunchKernelGGL(k_jb_bb_box<DD>, dim3(g), dim3(256), 0, st, P, bt, nbt, HT, t->isn.as<uint32_t>(),       \
                           t->offn.as<uint32_t>(), nbase, (uint32_t)d);
    if (t->D == 2) {
        PSI_JBW(2)
    } else {
        PSI_JBW(3)
    }
#undef PSI_JBW
    return hip_ok(hipGetLastError());
}

// One batch update, run again with larger pools if one ran out. del: the
// batch is the (key, id) pairs of live entries to remove, else new entries
// with their points.
psi_status jb_update(psi_bst t, bool del, const uint64_t* bk, const uint32_t* bi, const uint32_t* bp, uint32_t m) {
    hipStream_t st = t->ix->st;
    psi_status s;
    const uint64_t est = (uint64_t)m / std::max<uint32_t>(t->phi / 4, 1) + 64;
    uint64_t want_n = (uint64_t)t->nbump + 2 * est, want_l = (uint64_t)t->lbump + 2 * est;
    if ((s = t->ctr.ensure(C_COUNT * 4)) != PSI_OK) return s;
    for (int attempt = 0; attempt < 12; ++attempt) {
        if ((s = jb_grow(t, want_n, want_l)) != PSI_OK) return s;
        uint32_t h[C_COUNT] = {};
        h[C_NBUMP] = t->nbump;
        h[C_LBUMP] = t->lbump;
        h[C_ROOT] = JB_NIL;
        if ((s = jb_set_counters(t, h)) != PSI_OK) return s;
        if ((s = t->task[0].ensure(sizeof(JTask))) != PSI_OK) return s;
        const JTask t0{t->root, 0u, m, JB_NIL};
        if ((s = hip_ok(hipMemcpy(t->task[0].p, &t0, sizeof t0, hipMemcpyHostToDevice))) != PSI_OK) return s;
        std::vector<uint32_t> rec_start;
        uint32_t nt = 1, recs = 0, bigs = 0;
        bool overflow = false;
        int level = 0;
        while (nt > 0) {
            if (++level > 4096) return PSI_E_INTERNAL;
            const int cur = (level - 1) & 1, nxt = level & 1;
            if ((s = t->task[nxt].ensure((uint64_t)2 * nt * sizeof(JTask))) != PSI_OK) return s;
            if ((s = t->rec.grow_keep(((uint64_t)recs + nt + 1) * sizeof(JRec), (uint64_t)recs * sizeof(JRec), st)) !=
                PSI_OK)
                return s;
            if (!del &&
                (s = t->big.grow_keep(((uint64_t)bigs + nt + 1) * sizeof(JTask), (uint64_t)bigs * sizeof(JTask), st)) !=
                    PSI_OK)
                return s;
            h[C_TASKS] = 0;
            launch_fill_u32(st, t->ctr.as<uint32_t>() + C_TASKS, 1, 0u);
            const Pools P = jb_pools(t, bk, bi, bp, m);
            const unsigned g = blocks_of(nt, 64);
            const uint32_t tcap = 2 * nt;
            const uint32_t bcap = (uint32_t)std::min<uint64_t>(t->big.bytes / sizeof(JTask), 1u << 30);
            if (del) {
                if (t->D == 2)
                    hipLaunchKernelGGL(k_jb_del_down<2>, dim3(g), dim3(64), 0, st, P, t->task[cur].as<JTask>(), nt,
                                       t->task[nxt].as<JTask>(), tcap);
                else
                    hipLaunchKernelGGL(k_jb_del_down<3>, dim3(g), dim3(64), 0, st, P, t->task[cur].as<JTask>(), nt,
                                       t->task[nxt].as<JTask>(), tcap);
            } else {
                if (t->D == 2)
                    hipLaunchKernelGGL(k_jb_ins_down<2>, dim3(g), dim3(64), 0, st, P, t->task[cur].as<JTask>(), nt,
                                       t->task[nxt].as<JTask>(), tcap, t->big.as<JTask>(), bcap);
                else
                    hipLaunchKernelGGL(k_jb_ins_down<3>, dim3(g), dim3(64), 0, st, P, t->task[cur].as<JTask>(), nt,
                                       t->task[nxt].as<JTask>(), tcap, t->big.as<JTask>(), bcap);
            }
            if ((s = hip_ok(hipGetLastError())) != PSI_OK) return s;
            if ((s = jb_counters(t, h)) != PSI_OK) return s;
            rec_start.push_back(recs);
            if (h[C_FLAGS] & F_OVERFLOW) {
                overflow = true;
                break;
            }
            nt = h[C_TASKS];
            recs = h[C_RECS];
            bigs = h[C_BIG];
        }
        if (!overflow) {
            rec_start.push_back(recs);
            if (bigs) {
                std::vector<JTask> bl(bigs);
                if ((s = hip_ok(hipMemcpy(bl.data(), t->big.p, (size_t)bigs * sizeof(JTask), hipMemcpyDeviceToHost))) !=
                    PSI_OK)
                    return s;
                if ((s = jb_big_builds(t, bl, bk, bi, bp, m, h)) != PSI_OK) return s;
            }
            const Pools P = jb_pools(t, bk, bi, bp, m);
            for (int lv = (int)rec_start.size() - 2; lv >= 0; --lv) {
                const uint32_t r0 = rec_start[lv], r1 = rec_start[lv + 1];
                if (r1 <= r0) continue;
                const unsigned g = blocks_of(r1 - r0, 64);
                if (t->D == 2) hipLaunchKernelGGL(k_jb_up<2>, dim3(g), dim3(64), 0, st, P, r0, r1);
                else hipLaunchKernelGGL(k_jb_up<3>, dim3(g), dim3(64), 0, st, P, r0, r1);
            }
            if ((s = hip_ok(hipGetLastError())) != PSI_OK) return s;
            if ((s = jb_counters(t, h)) != PSI_OK) return s;
            overflow = (h[C_FLAGS] & F_OVERFLOW) != 0;
        }
        if (overflow) {  // nothing reachable from the root changed: grow and run again
            want_n = (uint64_t)std::max(t->ncap, 16u) * 2;
            want_l = (uint64_t)std::max(t->lcap, 16u) * 2;
            continue;
        }
        if (h[C_FLAGS] & F_BROKEN) return PSI_E_INTERNAL;
        // commit
        const uint32_t ntake = std::min(h[C_NTAKE], t->nfree_n), ltake = std::min(h[C_LTAKE], t->lfree_n);
        const uint32_t nkeep = t->nfree_n - ntake, lkeep = t->lfree_n - ltake;
        const uint32_t nc = h[C_NCONS], lc = h[C_LCONS];
        if ((uint64_t)nkeep + nc > t->ncap || (uint64_t)lkeep + lc > t->lcap) return PSI_E_INTERNAL;
        hipLaunchKernelGGL(k_jb_commit, dim3(blocks_of(std::max(nc, lc), 256)), dim3(256), 0, st,
                           t->nfree.as<uint32_t>(), nkeep, t->ncons.as<uint32_t>(), nc, t->lfree.as<uint32_t>(), lkeep,
                           t->lcons.as<uint32_t>(), lc);
        if ((s = hip_ok(hipGetLastError())) != PSI_OK) return s;
        t->nfree_n = nkeep + nc;
        t->lfree_n = lkeep + lc;
        t->nbump = std::min(h[C_NBUMP], t->ncap);
        t->lbump = std::min(h[C_LBUMP], t->lcap);
        t->root = h[C_ROOT];
        return hip_ok(hipStreamSynchronize(st));
    }
    return PSI_E_NOMEM;
}

void jb_gather(psi_bst t, const uint32_t* ids, uint64_t n, const uint32_t* src, uint32_t id_base, uint32_t* out) {
    if (!n) return;
    const unsigned g = blocks_of(n, 256);
    if (t->D == 2) hipLaunchKernelGGL(k_jb_gather<2>, dim3(g), dim3(256), 0, t->ix->st, ids, n, src, id_base, out);
    else hipLaunchKernelGGL(k_jb_gather<3>, dim3(g), dim3(256), 0, t->ix->st, ids, n, src, id_base, out);
}

// Per-id tables grown to cover ids below upto (contents kept).
psi_status jb_ids(psi_bst t, uint64_t upto) {
    psi_status s = t->alive.grow_keep(std::max<uint64_t>(upto, 1) * 4, t->alive.bytes, t->ix->st);
    if (s == PSI_OK) s = t->idkey.grow_keep(std::max<uint64_t>(upto, 1) * 8, t->idkey.bytes, t->ix->st);
    return s;
}

// Encodes and sorts m points with ids base .. base + m - 1: their keys go to
// the id -> key table, the sorted pairs to the sorter (*w), the points in
// sorted order to bpts.
psi_status jb_encode(psi_bst t, const uint32_t* d_pts, uint64_t m, uint32_t base, int* w) {
    psi_status s;
    if ((s = t->kin.ensure(m * 8)) != PSI_OK) return s;
    if ((s = t->bpts.ensure(m * 4 * t->D)) != PSI_OK) return s;
    if ((s = encode_sort(t->ix, d_pts, m, t->kin.as<uint64_t>(), base, w)) != PSI_OK) return s;
    hipLaunchKernelGGL(k_jb_copy_u64, dim3(blocks_of(m, 256)), dim3(256), 0, t->ix->st,
                       t->idkey.as<uint64_t>() + base, t->kin.as<uint64_t>(), m);
    jb_gather(t, t->ix->sorter.i[*w].as<uint32_t>(), m, d_pts, base, t->bpts.as<uint32_t>());
    return hip_ok(hipGetLastError());
}

}  // namespace

extern "C" {

psi_status psi_bst_create(uint32_t dim, uint32_t curve, uint32_t leaf_wrap, void* hip_stream, psi_bst* out) {
    if (!out || (dim != 2 && dim != 3) || curve > 1 || leaf_wrap < 2 || leaf_wrap > JB_PHI_MAX) return PSI_E_ARG;
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
    hipStream_t st = t->ix->st;
    t->n = 0;
    t->next_id = 0;
    t->root = JB_NIL;
    t->nbump = t->lbump = t->nfree_n = t->lfree_n = 0;
    if ((s = jb_ids(t, n)) != PSI_OK) return s;
    if ((s = t->ctr.ensure(C_COUNT * 4)) != PSI_OK) return s;
    int w = 0;
    const uint64_t* bk = nullptr;
    const uint32_t* bi = nullptr;
    if (n) {
        if ((s = jb_encode(t, d_pts, n, 0, &w)) != PSI_OK) return s;
        bk = t->ix->sorter.k[w].as<uint64_t>();
        bi = t->ix->sorter.i[w].as<uint32_t>();
        hipLaunchKernelGGL(k_jb_fill, dim3(blocks_of(n, 256)), dim3(256), 0, st, t->alive.as<uint32_t>(), 0ull, n, 1u);
    }
    if ((s = psi_sync(t->ix)) != PSI_OK) return s;  // an out-of-range point fails the build here
    uint32_t h[C_COUNT] = {};
    h[C_ROOT] = JB_NIL;
    if ((s = jb_set_counters(t, h)) != PSI_OK) return s;
    std::vector<JTask> one(1, JTask{JB_NIL, 0u, (uint32_t)n, JB_NIL});
    if ((s = jb_big_builds(t, one, bk, bi, t->bpts.as<uint32_t>(), (uint32_t)n, h)) != PSI_OK) return s;
    if ((s = jb_counters(t, h)) != PSI_OK) return s;
    if (h[C_FLAGS]) return PSI_E_INTERNAL;
    t->root = h[C_ROOT];
    t->nbump = h[C_NBUMP];
    t->lbump = h[C_LBUMP];
    t->n = n;
    t->next_id = (uint32_t)n;
    return psi_sync(t->ix);
}

psi_status psi_bst_batch_insert(psi_bst t, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids) {
    if (!t || (m && (!d_pts || !d_new_ids))) return PSI_E_ARG;
    if (m == 0) return PSI_OK;
    if ((uint64_t)t->next_id + m >= (1ull << 31)) return PSI_E_CAPACITY;
    if (capturing(t->ix->st)) return PSI_E_STATE;
    if (t->root == JB_NIL) return PSI_E_STATE;  // never built
    psi_status s;
    hipStream_t st = t->ix->st;
    const uint32_t base = t->next_id;
    if ((s = jb_ids(t, (uint64_t)base + m)) != PSI_OK) return s;
    int w = 0;
    if ((s = jb_encode(t, d_pts, m, base, &w)) != PSI_OK) return s;
    if ((s = psi_sync(t->ix)) != PSI_OK) return s;  // an out-of-range point rejects the batch
    const uint64_t* bk = t->ix->sorter.k[w].as<uint64_t>();
    const uint32_t* bi = t->ix->sorter.i[w].as<uint32_t>();
    if ((s = jb_update(t, false, bk, bi, t->bpts.as<uint32_t>(), (uint32_t)m)) != PSI_OK) return s;
    hipLaunchKernelGGL(k_jb_fill, dim3(blocks_of(m, 256)), dim3(256), 0, st, t->alive.as<uint32_t>(), (uint64_t)base,
                       (uint64_t)base + m, 1u);
    hipLaunchKernelGGL(k_jb_iota, dim3(blocks_of(m, 256)), dim3(256), 0, st, d_new_ids, m, base);
    t->n += m;
    t->next_id = base + (uint32_t)m;
    return psi_sync(t->ix);
}

psi_status psi_bst_batch_delete(psi_bst t, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted) {
    if (!t || (m && !d_ids)) return PSI_E_ARG;
    if (capturing(t->ix->st)) return PSI_E_STATE;
    psi_status s;
    hipStream_t st = t->ix->st;
    if ((s = t->nd.ensure(8)) != PSI_OK) return s;
    if ((s = t->dk.ensure(std::max<uint64_t>(m, 1) * 8)) != PSI_OK) return s;
    if ((s = t->di.ensure(std::max<uint64_t>(m, 1) * 4)) != PSI_OK) return s;
    launch_fill_u32(st, t->nd.as<uint32_t>(), 2, 0u);
    if (m && t->next_id)
        hipLaunchKernelGGL(k_jb_claim, dim3(blocks_of(m, 256)), dim3(256), 0, st, d_ids, m, t->next_id,
                           t->alive.as<uint32_t>(), t->idkey.as<uint64_t>(), t->dk.as<uint64_t>(),
                           t->di.as<uint32_t>(), t->nd.as<unsigned long long>());
    if (d_ndeleted &&
        (s = hip_ok(hipMemcpyAsync(d_ndeleted, t->nd.p, 8, hipMemcpyDeviceToDevice, st))) != PSI_OK)
        return s;
    if ((s = readback(t->ix, t->nd.p, 8)) != PSI_OK) return s;
    uint64_t md = 0;
    std::memcpy(&md, t->ix->pinned, 8);
    if (md == 0) return psi_sync(t->ix);
    int w = 0;
    if ((s = sort_pairs(t->ix, t->dk.as<uint64_t>(), t->di.as<uint32_t>(), 0, md, true, false, &w, "bst_sort")) !=
        PSI_OK)
        return s;
    const uint64_t* bk = t->ix->sorter.k[w].as<uint64_t>();
    const uint32_t* bi = t->ix->sorter.i[w].as<uint32_t>();
    if ((s = jb_update(t, true, bk, bi, nullptr, (uint32_t)md)) != PSI_OK) return s;
    t->n -= md;
    return psi_sync(t->ix);
}

psi_status psi_bst_knn(psi_bst t, const uint32_t* d_q, uint64_t nq, uint32_t k, uint32_t* d_ids, uint64_t* d_d2) {
    if (!t || k == 0 || k > 16 || (nq && (!d_q || !d_ids || !d_d2))) return PSI_E_ARG;
    if (nq == 0) return PSI_OK;
    const uint32_t* order = nullptr;
    psi_status s = query_order(t->ix, d_q, nq, false, &order);
    if (s != PSI_OK) return s;
    const JView v = jb_view(t);
    const unsigned g = (unsigned)((nq + JB_QT - 1) / JB_QT);
    hipStream_t st = t->ix->st;
    uint32_t* err = t->ix->err.as<uint32_t>();
#define PSI_BK(DD, KK) \
    hipLaunchKernelGGL((k_jb_knn<DD, KK>), dim3(g), dim3(JB_QT), 0, st, v, d_q, nq, order, d_ids, d_d2, err)
#define PSI_BK_ALL(DD)                                                                                       \
    switch (k) {                                                                                             \
        case 1: PSI_BK(DD, 1); break;   case 2: PSI_BK(DD, 2); break;   case 3: PSI_BK(DD, 3); break;        \
        case 4: PSI_BK(DD, 4); break;   case 5: PSI_BK(DD, 5); break;   case 6: PSI_BK(DD, 6); break;        \
        case 7: PSI_BK(DD, 7); break;   case 8: PSI_BK(DD, 8); break;   case 9: PSI_BK(DD, 9); break;        \
        case 10: PSI_BK(DD, 10); break; case 11: PSI_BK(DD, 11); break; case 12: PSI_BK(DD, 12); break;      \
        case 13: PSI_BK(DD, 13); break; case 14: PSI_BK(DD, 14); break; case 15: PSI_BK(DD, 15); break;      \
        default: PSI_BK(DD, 16); break;                                                                      \
    }
    if (t->D == 2) {
        PSI_BK_ALL(2)
    } else {
        PSI_BK_ALL(3)
    }
#undef PSI_BK_ALL
#undef PSI_BK
    return hip_ok(hipGetLastError());
}

static psi_status jb_range(psi_bst t, const uint32_t* d_boxes, uint64_t nb, uint64_t* d_counts,
                           const uint64_t* d_offsets, uint32_t* d_ids, bool report) {
    const uint32_t* order = nullptr;
    psi_status s = query_order(t->ix, d_boxes, nb, true, &order);
    if (s != PSI_OK) return s;
    const JView v = jb_view(t);
    const unsigned g = (unsigned)((nb + JB_QT - 1) / JB_QT);
    hipStream_t st = t->ix->st;
    uint32_t* err = t->ix->err.as<uint32_t>();
    if (t->D == 2) {
        if (report)
            hipLaunchKernelGGL((k_jb_range<2, true>), dim3(g), dim3(JB_QT), 0, st, v, d_boxes, nb, order, nullptr,
                               d_offsets, d_ids, err);
        else
            hipLaunchKernelGGL((k_jb_range<2, false>), dim3(g), dim3(JB_QT), 0, st, v, d_boxes, nb, order, d_counts,
                               nullptr, nullptr, err);
    } else {
        if (report)
            hipLaunchKernelGGL((k_jb_range<3, true>), dim3(g), dim3(JB_QT), 0, st, v, d_boxes, nb, order, nullptr,
                               d_offsets, d_ids, err);
        else
            hipLaunchKernelGGL((k_jb_range<3, false>), dim3(g), dim3(JB_QT), 0, st, v, d_boxes, nb, order, d_counts,
                               nullptr, nullptr, err);
    }
    return hip_ok(hipGetLastError());
}

psi_status psi_bst_range_count(psi_bst t, const uint32_t* d_boxes, uint64_t nb, uint64_t* d_counts) {
    if (!t || (nb && (!d_boxes || !d_counts))) return PSI_E_ARG;
    if (nb == 0) return PSI_OK;
    return jb_range(t, d_boxes, nb, d_counts, nullptr, nullptr, false);
}

psi_status psi_bst_range_report(psi_bst t, const uint32_t* d_boxes, uint64_t nb, const uint64_t* d_offsets,
                                uint32_t* d_ids) {
    if (!t || (nb && (!d_boxes || !d_offsets))) return PSI_E_ARG;
    if (nb == 0) return PSI_OK;
    return jb_range(t, d_boxes, nb, nullptr, d_offsets, d_ids, true);
}

psi_status psi_bst_sync(psi_bst t) {
    if (!t) return PSI_E_ARG;
    return psi_sync(t->ix);
}

psi_status psi_bst_shape(psi_bst t, uint64_t* h_n, uint32_t* h_root, uint64_t* h_node_slots,
                         uint64_t* h_leaf_slots) {
    if (!t || !h_n || !h_root || !h_node_slots || !h_leaf_slots) return PSI_E_ARG;
    psi_status s = psi_sync(t->ix);
    if (s != PSI_OK) return s;
    *h_n = t->n;
    *h_root = t->root;
    *h_node_slots = t->nbump;
    *h_leaf_slots = t->lbump;
    return PSI_OK;
}

psi_status psi_bst_export(psi_bst t, uint32_t* d_nodes, uint32_t* d_leaves, uint32_t* d_ids, uint32_t* d_pts) {
    if (!t || !d_nodes || !d_leaves || !d_ids || !d_pts) return PSI_E_ARG;
    hipStream_t st = t->ix->st;
    psi_status s = PSI_OK;
    const uint64_t phi = t->phi;
    if (t->nbump)
        s = hip_ok(hipMemcpyAsync(d_nodes, t->node.p, (size_t)t->nbump * sizeof(JNode), hipMemcpyDeviceToDevice, st));
    if (s == PSI_OK && t->lbump) {
        s = hip_ok(hipMemcpyAsync(d_leaves, t->leaf.p, (size_t)t->lbump * sizeof(JLeaf), hipMemcpyDeviceToDevice, st));
        if (s == PSI_OK)
            s = hip_ok(hipMemcpyAsync(d_ids, t->lid.p, (size_t)t->lbump * phi * 4, hipMemcpyDeviceToDevice, st));
        if (s == PSI_OK)
            s = hip_ok(
                hipMemcpyAsync(d_pts, t->lpt.p, (size_t)t->lbump * phi * 4 * t->D, hipMemcpyDeviceToDevice, st));
    }
    if (s != PSI_OK) return s;
    return psi_sync(t->ix);
}

}  // extern "C"
