// Plain CPU oracle for the SPaC-tree hot path ("Parallel Dynamic Spatial
// Indexes", PPoPP'26).
//
// TEST INFRASTRUCTURE ONLY. This file is a slow, obviously-correct statement
// of what the index computes. Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load it. It shares no code, header, table
// or helper with the HIP library, and it never calls into it.
//
// Parity status of every function: pinned (see tests/test_oracle_*.py):
//   morton / hilbert keys ........ closed-form values, bijection, unit-step,
//                                  nesting and prefix invariants
//   sort of (key,id) ............. sortedness + permutation
//   canonical leaves / nodes ..... closed form of the balanced chunking,
//                                  brute-force boxes and counts
//   insert / delete .............. set algebra identities
//   kNN / range .................. hand lattices, second brute force
//
// Conventions (readings of passages the paper leaves open):
//   * Morton key (Sec. 2.2 "Spatial Filling Curves"): bit b of coordinate d
//     goes to key bit D*b + d (x in the least significant bit of each group).
//   * Hilbert key (Sec. 2.2): Skilling's transpose construction (J. Skilling,
//     "Programming the Hilbert curve", AIP Conf. Proc. 707, 2004) with the
//     order fixed at W = 32 bits per axis in 2D and W = 21 in 3D, the widths
//     a 64-bit key allows (Sec. 3, SFC precision limits).
//   * (key, id) pairs are ordered lexicographically; ids break key ties
//     (equal keys only arise from duplicate points).
//   * Leaves of a fresh build are L = ceil(n / phi) balanced consecutive
//     chunks of the sorted pairs; nodes form a B-ary tree over the leaves
//     with left-packed levels (Alg. 3 BuildSorted, done bottom-up).
//   * kNN (Sec. 2.2 "Queries"): the k points with the smallest
//     (squared Euclidean distance, id); rows padded with
//     (0xFFFFFFFF, UINT64_MAX) when fewer than k points exist.
//   * Range queries (Sec. 2.2): closed boxes lo <= p <= hi in every axis; a
//     box with lo > hi in any axis is empty.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <queue>
#include <thread>
#include <utility>
#include <vector>

namespace {

const uint32_t kPadId = 0xFFFFFFFFu;
const uint64_t kPadD2 = ~0ull;

int key_bits_per_axis(int dim) { return dim == 2 ? 32 : 21; }

// ------------------------------------------------------------------ C.1
// Morton (Z-order) key: interleave coordinate bits (Sec. 2.2).
uint64_t morton_key(int dim, const uint32_t* p) {
    const int W = key_bits_per_axis(dim);
    uint64_t key = 0;
    for (int b = 0; b < W; ++b)
        for (int d = 0; d < dim; ++d)
            key |= (uint64_t)((p[d] >> b) & 1u) << (dim * b + d);
    return key;
}

// ------------------------------------------------------------------ C.2
// Hilbert key (Sec. 2.2) by Skilling's construction: turn the axes into the
// "transposed" Hilbert index, then read its bits from the top plane down,
// axis 0 first inside every plane.
uint64_t hilbert_key(int dim, const uint32_t* p) {
    const int W = key_bits_per_axis(dim);
    uint32_t X[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) X[d] = p[d];
    // (i) undo the excess reflections and exchanges, top plane first
    for (uint32_t Q = 1u << (W - 1); Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < dim; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;                       // reflect the low bits of axis 0
            } else {
                uint32_t t = (X[0] ^ X[i]) & P;  // exchange low bits of axis 0 and axis i
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    // (ii) Gray-code the planes
    for (int i = 1; i < dim; ++i) X[i] ^= X[i - 1];
    uint32_t t = 0;
    for (uint32_t Q = 1u << (W - 1); Q > 1; Q >>= 1)
        if (X[dim - 1] & Q) t ^= Q - 1;
    for (int i = 0; i < dim; ++i) X[i] ^= t;
    // (iii) read the transposed index plane by plane, most significant first
    uint64_t key = 0;
    for (int b = W - 1; b >= 0; --b)
        for (int i = 0; i < dim; ++i) key = (key << 1) | ((X[i] >> b) & 1u);
    return key;
}

uint64_t sfc_key(int dim, int curve, const uint32_t* p) {
    return curve == 0 ? morton_key(dim, p) : hilbert_key(dim, p);
}

bool coords_ok(int dim, const uint32_t* p) {
    const uint32_t lim = dim == 2 ? (1u << 31) : (1u << 21);
    for (int d = 0; d < dim; ++d)
        if (p[d] >= lim) return false;
    return true;
}

struct Entry {
    uint64_t key;
    uint32_t id;
    uint32_t p[3];
};

bool entry_less(const Entry& a, const Entry& b) {
    return a.key < b.key || (a.key == b.key && a.id < b.id);
}

uint64_t sq_dist(int dim, const uint32_t* a, const uint32_t* b) {
    uint64_t s = 0;
    for (int d = 0; d < dim; ++d) {
        uint64_t diff = a[d] > b[d] ? (uint64_t)(a[d] - b[d]) : (uint64_t)(b[d] - a[d]);
        s += diff * diff;
    }
    return s;
}

struct Index {
    int dim = 2;
    int curve = 0;
    uint32_t phi = 32;
    uint32_t fanout = 2;
    uint32_t next_id = 0;
    std::vector<Entry> S;       // live entries in (key, id) order
    std::vector<uint8_t> live;  // live[id]
};

template <class F>
void parallel_for(uint64_t n, int threads, F f) {
    if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
    if ((uint64_t)threads > n) threads = (int)std::max<uint64_t>(1, n);
    if (threads == 1) {
        for (uint64_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([=, &f] {
            for (uint64_t i = t; i < n; i += threads) f(i);
        });
    for (auto& th : pool) th.join();
}

// Canonical leaf chunking of a fresh build (bottom-up form of Alg. 3
// BuildSorted): L = ceil(n/phi) leaves, leaf j = S[floor(j n / L),
// floor((j+1) n / L)).
uint64_t num_leaves(uint64_t n, uint32_t phi) { return n == 0 ? 0 : (n + phi - 1) / phi; }
uint64_t leaf_begin(uint64_t j, uint64_t n, uint64_t L) { return j * n / L; }

// Height h of the B-ary tree over L leaves: smallest h with B^h >= L.
uint32_t tree_height(uint64_t L, uint32_t B) {
    uint32_t h = 0;
    uint64_t span = 1;
    while (span < L) { span *= B; ++h; }
    return h;
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------- keys, sort
uint64_t ora_morton(int dim, const uint32_t* p) { return morton_key(dim, p); }
uint64_t ora_hilbert(int dim, const uint32_t* p) { return hilbert_key(dim, p); }

void ora_encode(int dim, int curve, const uint32_t* pts, uint64_t n, uint64_t* keys) {
    for (uint64_t i = 0; i < n; ++i) keys[i] = sfc_key(dim, curve, pts + i * dim);
}

// Sort (key, id) pairs lexicographically in place (Alg. 3 sorts only the
// (code, id) pairs, never the coordinates).
void ora_sort_pairs(uint64_t n, uint64_t* keys, uint32_t* ids) {
    std::vector<std::pair<uint64_t, uint32_t>> v(n);
    for (uint64_t i = 0; i < n; ++i) v[i] = {keys[i], ids[i]};
    std::sort(v.begin(), v.end());
    for (uint64_t i = 0; i < n; ++i) { keys[i] = v[i].first; ids[i] = v[i].second; }
}

// ------------------------------------------------------------------ index
void* ora_new(int dim, int curve, uint32_t phi, uint32_t fanout) {
    if ((dim != 2 && dim != 3) || (curve != 0 && curve != 1) || phi < 2 || fanout < 2) return nullptr;
    Index* x = new Index;
    x->dim = dim; x->curve = curve; x->phi = phi; x->fanout = fanout;
    return x;
}

void ora_free(void* h) { delete static_cast<Index*>(h); }

// Build (Alg. 3): encode every point, sort (code, id), keep the sorted set.
// Returns 0, or -1 if a coordinate is out of range (nothing changes then).
int ora_build(void* h, const uint32_t* pts, uint64_t n) {
    Index* x = static_cast<Index*>(h);
    for (uint64_t i = 0; i < n; ++i)
        if (!coords_ok(x->dim, pts + i * x->dim)) return -1;
    x->S.resize(n);
    for (uint64_t i = 0; i < n; ++i) {
        Entry& e = x->S[i];
        std::memset(e.p, 0, sizeof e.p);
        std::memcpy(e.p, pts + i * x->dim, sizeof(uint32_t) * x->dim);
        e.id = (uint32_t)i;
        e.key = sfc_key(x->dim, x->curve, e.p);
    }
    std::sort(x->S.begin(), x->S.end(), entry_less);
    x->next_id = (uint32_t)n;
    x->live.assign(n, 1);
    return 0;
}

// Batch insert (Alg. 4): the new points get ids next_id, next_id+1, ... in
// input order; the set becomes S united with the new (key, id) entries.
int ora_insert(void* h, const uint32_t* pts, uint64_t m, uint32_t* new_ids) {
    Index* x = static_cast<Index*>(h);
    for (uint64_t i = 0; i < m; ++i)
        if (!coords_ok(x->dim, pts + i * x->dim)) return -1;
    if ((uint64_t)x->next_id + m > 0xFFFFFFFFull) return -2;
    std::vector<Entry> B(m);
    for (uint64_t i = 0; i < m; ++i) {
        Entry& e = B[i];
        std::memset(e.p, 0, sizeof e.p);
        std::memcpy(e.p, pts + i * x->dim, sizeof(uint32_t) * x->dim);
        e.id = x->next_id + (uint32_t)i;
        e.key = sfc_key(x->dim, x->curve, e.p);
        if (new_ids) new_ids[i] = e.id;
    }
    std::sort(B.begin(), B.end(), entry_less);
    std::vector<Entry> out(x->S.size() + m);
    std::merge(x->S.begin(), x->S.end(), B.begin(), B.end(), out.begin(), entry_less);
    x->S.swap(out);
    x->next_id += (uint32_t)m;
    x->live.resize(x->next_id, 1);
    return 0;
}

// Batch delete (Sec. 4.2): remove the entries whose id is in the batch and
// still live. Unknown, dead and repeated ids are ignored. Returns the number
// of entries removed.
uint64_t ora_delete(void* h, const uint32_t* ids, uint64_t m) {
    Index* x = static_cast<Index*>(h);
    std::vector<uint8_t> kill(x->next_id, 0);
    uint64_t removed = 0;
    for (uint64_t i = 0; i < m; ++i) {
        uint32_t id = ids[i];
        if (id < x->next_id && x->live[id] && !kill[id]) { kill[id] = 1; ++removed; }
    }
    std::vector<Entry> out;
    out.reserve(x->S.size() - removed);
    for (const Entry& e : x->S)
        if (!kill[e.id]) out.push_back(e);
    x->S.swap(out);
    for (uint32_t id = 0; id < x->next_id; ++id)
        if (kill[id]) x->live[id] = 0;
    return removed;
}

uint64_t ora_size(void* h) { return static_cast<Index*>(h)->S.size(); }
uint32_t ora_next_id(void* h) { return static_cast<Index*>(h)->next_id; }

// Live entries in (key, id) order; pts is [n][dim].
void ora_dump(void* h, uint64_t* keys, uint32_t* ids, uint32_t* pts) {
    Index* x = static_cast<Index*>(h);
    for (uint64_t i = 0; i < x->S.size(); ++i) {
        const Entry& e = x->S[i];
        if (keys) keys[i] = e.key;
        if (ids) ids[i] = e.id;
        if (pts) std::memcpy(pts + i * x->dim, e.p, sizeof(uint32_t) * x->dim);
    }
}

// --------------------------------------------------- canonical structure
// Shape of the canonical structure of the current set: number of leaves,
// tree height h, and node count of every level 0..h (level h = leaves).
void ora_struct_shape(void* h, uint64_t* n_leaves, uint32_t* height, uint64_t* level_sizes) {
    Index* x = static_cast<Index*>(h);
    const uint64_t n = x->S.size();
    const uint64_t L = num_leaves(n, x->phi);
    *n_leaves = L;
    if (L == 0) { *height = 0; return; }
    const uint32_t hh = tree_height(L, x->fanout);
    *height = hh;
    for (uint32_t lev = 0; lev <= hh; ++lev) {
        uint64_t span = 1;
        for (uint32_t s = lev; s < hh; ++s) span *= x->fanout;
        level_sizes[lev] = (L + span - 1) / span;
    }
}

// Canonical leaves and nodes of the current set, as a fresh build lays them
// out. Leaf j: pivot = first (key, id) of its chunk, count, tight closed box.
// Node (level, i) covers leaves [i*B^(h-level), (i+1)*B^(h-level)) clipped to
// L; its box is the union and its count the sum over those leaves. Node
// arrays are level-major from the root (level 0) down to the leaves.
// Boxes are [node][dim] lo and hi arrays.
void ora_struct(void* h, uint64_t* piv_key, uint32_t* piv_id, uint32_t* leaf_cnt,
                uint32_t* leaf_lo, uint32_t* leaf_hi,
                uint32_t* node_lo, uint32_t* node_hi, uint64_t* node_cnt) {
    Index* x = static_cast<Index*>(h);
    const int D = x->dim;
    const uint64_t n = x->S.size();
    const uint64_t L = num_leaves(n, x->phi);
    if (L == 0) return;
    for (uint64_t j = 0; j < L; ++j) {
        const uint64_t b = leaf_begin(j, n, L), e = leaf_begin(j + 1, n, L);
        piv_key[j] = x->S[b].key;
        piv_id[j] = x->S[b].id;
        leaf_cnt[j] = (uint32_t)(e - b);
        for (int d = 0; d < D; ++d) {
            uint32_t lo = 0xFFFFFFFFu, hi = 0;
            for (uint64_t i = b; i < e; ++i) {
                lo = std::min(lo, x->S[i].p[d]);
                hi = std::max(hi, x->S[i].p[d]);
            }
            leaf_lo[j * D + d] = lo;
            leaf_hi[j * D + d] = hi;
        }
    }
    const uint32_t hh = tree_height(L, x->fanout);
    uint64_t base = 0;
    for (uint32_t lev = 0; lev <= hh; ++lev) {
        uint64_t span = 1;
        for (uint32_t s = lev; s < hh; ++s) span *= x->fanout;
        const uint64_t N = (L + span - 1) / span;
        for (uint64_t i = 0; i < N; ++i) {
            const uint64_t j0 = i * span, j1 = std::min(L, (i + 1) * span);
            uint64_t cnt = 0;
            for (int d = 0; d < D; ++d) {
                node_lo[(base + i) * D + d] = 0xFFFFFFFFu;
                node_hi[(base + i) * D + d] = 0;
            }
            for (uint64_t j = j0; j < j1; ++j) {
                cnt += leaf_cnt[j];
                for (int d = 0; d < D; ++d) {
                    node_lo[(base + i) * D + d] = std::min(node_lo[(base + i) * D + d], leaf_lo[j * D + d]);
                    node_hi[(base + i) * D + d] = std::max(node_hi[(base + i) * D + d], leaf_hi[j * D + d]);
                }
            }
            node_cnt[base + i] = cnt;
        }
        base += N;
    }
}

// ---------------------------------------------------------------- queries
// k nearest neighbours (Sec. 2.2) by brute force: every live point is scored
// by (squared distance, id) and the k smallest are kept, ascending.
void ora_knn(void* h, const uint32_t* q, uint64_t nq, uint32_t k, uint32_t* out_ids,
             uint64_t* out_d2, int threads) {
    Index* x = static_cast<Index*>(h);
    const int D = x->dim;
    parallel_for(nq, threads, [&](uint64_t qi) {
        const uint32_t* qq = q + qi * D;
        std::priority_queue<std::pair<uint64_t, uint32_t>> best;  // max-heap of the k smallest
        for (const Entry& e : x->S) {
            std::pair<uint64_t, uint32_t> c{sq_dist(D, e.p, qq), e.id};
            if (best.size() < k) best.push(c);
            else if (k > 0 && c < best.top()) { best.pop(); best.push(c); }
        }
        std::vector<std::pair<uint64_t, uint32_t>> r;
        while (!best.empty()) { r.push_back(best.top()); best.pop(); }
        std::reverse(r.begin(), r.end());
        for (uint32_t j = 0; j < k; ++j) {
            out_ids[qi * k + j] = j < r.size() ? r[j].second : kPadId;
            out_d2[qi * k + j] = j < r.size() ? r[j].first : kPadD2;
        }
    });
}

// Second, independent brute force used to pin ora_knn: full sort of all
// (squared distance, id) pairs.
void ora_knn_fullsort(void* h, const uint32_t* q, uint64_t nq, uint32_t k, uint32_t* out_ids,
                      uint64_t* out_d2) {
    Index* x = static_cast<Index*>(h);
    const int D = x->dim;
    for (uint64_t qi = 0; qi < nq; ++qi) {
        std::vector<std::pair<uint64_t, uint32_t>> all;
        for (const Entry& e : x->S) all.push_back({sq_dist(D, e.p, q + qi * D), e.id});
        std::sort(all.begin(), all.end());
        for (uint32_t j = 0; j < k; ++j) {
            out_ids[qi * k + j] = j < all.size() ? all[j].second : kPadId;
            out_d2[qi * k + j] = j < all.size() ? all[j].first : kPadD2;
        }
    }
}

static bool in_box(int D, const uint32_t* p, const uint32_t* box) {
    for (int d = 0; d < D; ++d)
        if (p[d] < box[d] || p[d] > box[D + d]) return false;
    return true;
}

// Range count (Sec. 2.2): number of live points in the closed box.
// Boxes are [nb][2][dim]: lo row then hi row.
void ora_range_count(void* h, const uint32_t* boxes, uint64_t nb, uint64_t* counts, int threads) {
    Index* x = static_cast<Index*>(h);
    const int D = x->dim;
    parallel_for(nb, threads, [&](uint64_t b) {
        uint64_t c = 0;
        for (const Entry& e : x->S) c += in_box(D, e.p, boxes + b * 2 * D);
        counts[b] = c;
    });
}

// Range list (Sec. 2.2): ids of the live points in the box, ascending, written
// to ids[offsets[b] .. offsets[b+1]).
void ora_range_report(void* h, const uint32_t* boxes, uint64_t nb, const uint64_t* offsets,
                      uint32_t* ids, int threads) {
    Index* x = static_cast<Index*>(h);
    const int D = x->dim;
    parallel_for(nb, threads, [&](uint64_t b) {
        std::vector<uint32_t> r;
        for (const Entry& e : x->S)
            if (in_box(D, e.p, boxes + b * 2 * D)) r.push_back(e.id);
        std::sort(r.begin(), r.end());
        for (uint64_t i = 0; i < r.size() && offsets[b] + i < offsets[b + 1]; ++i) ids[offsets[b] + i] = r[i];
    });
}

// Brute-force kNN over a plain point array whose ids are 0..n-1 (used to
// check sampled queries against very large inputs without building a set).
void ora_knn_points(int dim, const uint32_t* pts, uint64_t n, const uint32_t* q, uint64_t nq, uint32_t k,
                    uint32_t* out_ids, uint64_t* out_d2, int threads) {
    parallel_for(nq, threads, [&](uint64_t qi) {
        const uint32_t* qq = q + qi * dim;
        std::priority_queue<std::pair<uint64_t, uint32_t>> best;
        for (uint64_t i = 0; i < n; ++i) {
            std::pair<uint64_t, uint32_t> c{sq_dist(dim, pts + i * dim, qq), (uint32_t)i};
            if (best.size() < k) best.push(c);
            else if (k > 0 && c < best.top()) { best.pop(); best.push(c); }
        }
        std::vector<std::pair<uint64_t, uint32_t>> r;
        while (!best.empty()) { r.push_back(best.top()); best.pop(); }
        std::reverse(r.begin(), r.end());
        for (uint32_t j = 0; j < k; ++j) {
            out_ids[qi * k + j] = j < r.size() ? r[j].second : kPadId;
            out_d2[qi * k + j] = j < r.size() ? r[j].first : kPadD2;
        }
    });
}

// Brute-force range count over a plain point array.
void ora_range_count_points(int dim, const uint32_t* pts, uint64_t n, const uint32_t* boxes, uint64_t nb,
                            uint64_t* counts, int threads) {
    parallel_for(nb, threads, [&](uint64_t b) {
        uint64_t c = 0;
        for (uint64_t i = 0; i < n; ++i) c += in_box(dim, pts + i * dim, boxes + b * 2 * dim);
        counts[b] = c;
    });
}

}  // extern "C"
