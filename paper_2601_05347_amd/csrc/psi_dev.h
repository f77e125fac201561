// Device-side building blocks of the gfx950 SPaC-tree library: record
// layouts, space-filling-curve keys (Sec. 2.2) and wave64 primitives.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PSI_HD __host__ __device__ __forceinline__

namespace psi {

// Error bits latched by kernels into the index's device error word.
enum : uint32_t {
    ERR_RANGE = 1u,     // a coordinate is out of the key's range
    ERR_SPIN = 2u,      // a bounded wait in the radix look-back gave up
    ERR_DELETE = 4u,    // a routed delete did not find its id in the leaf
    ERR_CAPACITY = 8u,  // a leaf slot overflowed (internal check)
    ERR_ORTH = 16u,     // a consistency check of the P-Orth build failed
    ERR_STACK = 32u,    // a kNN walk met a tree taller than its stack (internal check)
};

constexpr uint32_t PAD_ID = 0xFFFFFFFFu;
constexpr uint64_t PAD_D2 = ~0ull;
constexpr uint64_t DEAD_KEY = ~0ull;  // id-table entry of a deleted or unused id

// A node of the tree, leaves included (32 bytes). Boxes are closed; an empty
// node has lo = 0xFFFFFFFF, hi = 0 and cnt = 0. `slot` is the leaf's storage
// slot at the leaf level and unused above it; cnt and slot share one 8-byte
// word (what a leaf scan needs).
struct alignas(16) NodeRec {
    uint32_t lo[3];
    uint32_t hi[3];
    uint32_t cnt;
    uint32_t slot;
};

// A node's box in 16 bytes, for the kNN box tests (one 16-byte load each):
// the low corner in the first 64-bit word, the high corner in the second,
// axis d at bit d * W (W = 21 in 3D, 31 in 2D: coordinates are below 2^W,
// so the box is exact). Bit 63 of the first word marks an empty node.
template <int D> struct BoxBits { static constexpr int W = D == 2 ? 31 : 21; };
template <int D> PSI_HD void pack_box(const NodeRec& r, uint64_t& a, uint64_t& b) {
    a = 0;
    b = 0;
    for (int d = 0; d < D; ++d) {
        a |= (uint64_t)r.lo[d] << (d * BoxBits<D>::W);
        b |= (uint64_t)r.hi[d] << (d * BoxBits<D>::W);
    }
    if (r.cnt == 0) {
        a = 1ull << 63;
        b = 0;
    }
}
template <int D> PSI_HD uint4 packed_box(const NodeRec& r) {
    uint64_t a, b;
    pack_box<D>(r, a, b);
    return make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
}

// Node levels of the B-ary tree: level l (0 = root) has n[l] nodes stored at
// inner[off[l] ..]; level h is the leaf directory itself.
struct LevelInfo {
    uint64_t off;   // first node of the level in the inner array
    uint64_t n;     // nodes in the level
    uint64_t span;  // leaves under one node of the level: B^(h - l)
};
constexpr int MAX_LEVELS = 40;

// ---------------------------------------------------------------- keys
// Bits per axis of a 64-bit key (Sec. 3: 32 bits in 2D, 21 bits in 3D).
template <int D> struct KeyBits { static constexpr int W = D == 2 ? 32 : 21; };

PSI_HD uint64_t spread2(uint32_t v) {  // bit b -> bit 2b
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}
PSI_HD uint32_t gather2(uint64_t x) {  // bit 2b -> bit b
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    return (uint32_t)x;
}
PSI_HD uint64_t spread3(uint32_t v) {  // bit b -> bit 3b (21 bits)
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}
PSI_HD uint32_t gather3(uint64_t x) {  // bit 3b -> bit b
    x &= 0x1249249249249249ull;
    x = (x | (x >> 2)) & 0x10C30C30C30C30C3ull;
    x = (x | (x >> 4)) & 0x100F00F00F00F00Full;
    x = (x | (x >> 8)) & 0x001F0000FF0000FFull;
    x = (x | (x >> 16)) & 0x001F00000000FFFFull;
    x = (x | (x >> 32)) & 0x00000000001FFFFFull;
    return (uint32_t)x;
}

// Morton (Z) key: axis d supplies bit D*b + d.
template <int D> PSI_HD uint64_t morton_key(const uint32_t* p) {
    if constexpr (D == 2) return spread2(p[0]) | (spread2(p[1]) << 1);
    else return spread3(p[0]) | (spread3(p[1]) << 1) | (spread3(p[2]) << 2);
}
template <int D> PSI_HD void morton_point(uint64_t k, uint32_t* p) {
    if constexpr (D == 2) { p[0] = gather2(k); p[1] = gather2(k >> 1); }
    else { p[0] = gather3(k); p[1] = gather3(k >> 1); p[2] = gather3(k >> 2); }
}

// Hilbert key, Skilling's construction at W bits per axis: the point is
// folded into the "transposed" index A (one word per axis), which is then
// read plane by plane from the top, axis 0 being the most significant bit of
// every D-bit group.
template <int D> PSI_HD uint64_t hilbert_key(const uint32_t* p) {
    constexpr int W = KeyBits<D>::W;
    uint32_t A[D];
#pragma unroll
    for (int d = 0; d < D; ++d) A[d] = p[d];
    for (int s = W - 1; s >= 1; --s) {
        const uint32_t q = 1u << s, low = q - 1u;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const bool on = (A[d] & q) != 0;
            const uint32_t x = (A[0] ^ A[d]) & low;  // bits to exchange
            const uint32_t a0 = on ? (A[0] ^ low) : (A[0] ^ x);
            if (d != 0) A[d] = on ? A[d] : (A[d] ^ x);
            A[0] = a0;
        }
    }
#pragma unroll
    for (int d = 1; d < D; ++d) A[d] ^= A[d - 1];
    uint32_t flip = 0;
    for (int s = W - 1; s >= 1; --s)
        if (A[D - 1] & (1u << s)) flip ^= (1u << s) - 1u;
#pragma unroll
    for (int d = 0; d < D; ++d) A[d] ^= flip;
    if constexpr (D == 2) return (spread2(A[0]) << 1) | spread2(A[1]);
    else return (spread3(A[0]) << 2) | (spread3(A[1]) << 1) | spread3(A[2]);
}

// Inverse of hilbert_key: unpack the transposed index, undo the Gray code,
// then replay the exchanges and reflections from the lowest plane upward.
template <int D> PSI_HD void hilbert_point(uint64_t k, uint32_t* p) {
    constexpr int W = KeyBits<D>::W;
    uint32_t A[D];
    if constexpr (D == 2) { A[0] = gather2(k >> 1); A[1] = gather2(k); }
    else { A[0] = gather3(k >> 2); A[1] = gather3(k >> 1); A[2] = gather3(k); }
    const uint32_t g = A[D - 1] >> 1;
#pragma unroll
    for (int d = D - 1; d >= 1; --d) A[d] ^= A[d - 1];
    A[0] ^= g;
    for (int s = 1; s < W; ++s) {
        const uint32_t q = 1u << s, low = q - 1u;
#pragma unroll
        for (int d = D - 1; d >= 0; --d) {
            const bool on = (A[d] & q) != 0;
            const uint32_t x = (A[0] ^ A[d]) & low;
            const uint32_t a0 = on ? (A[0] ^ low) : (A[0] ^ x);
            if (d != 0) A[d] = on ? A[d] : (A[d] ^ x);
            A[0] = a0;
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) p[d] = A[d];
}

template <int D, int CURVE> PSI_HD uint64_t sfc_key(const uint32_t* p) {
    if constexpr (CURVE == 0) return morton_key<D>(p);
    else return hilbert_key<D>(p);
}
template <int D, int CURVE> PSI_HD void sfc_point(uint64_t k, uint32_t* p) {
    if constexpr (CURVE == 0) morton_point<D>(k, p);
    else hilbert_point<D>(k, p);
}

template <int D> PSI_HD bool coord_ok(const uint32_t* p) {
    constexpr uint32_t lim = D == 2 ? (1u << 31) : (1u << 21);
    bool ok = true;
#pragma unroll
    for (int d = 0; d < D; ++d) ok = ok && p[d] < lim;
    return ok;
}

// (key, id) order used everywhere: lexicographic.
PSI_HD bool pair_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

// Squared Euclidean distance of two points (exact in u64 for coordinates in
// range: Sec. 2.2's metric, squared to stay in integers).
template <int D>
__device__ __forceinline__ uint64_t pt_dist(const uint32_t* q, const uint32_t* p) {
    uint64_t s = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const uint64_t x = q[d] > p[d] ? q[d] - p[d] : p[d] - q[d];
        s += x * x;
    }
    return s;
}

// Insert (d, id) into an ascending list of K pairs held in registers: the
// new pair is carried down the list, swapping places with every larger
// entry, so the largest falls off the end. Every step updates its entry in
// place (no second copy of the list is live).
template <int K>
__device__ __forceinline__ void topk_insert(uint64_t (&bd)[K], uint32_t (&bi)[K], uint64_t d, uint32_t id) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const bool lt = pair_less(d, id, bd[j], bi[j]);
        const uint64_t od = bd[j];
        const uint32_t oi = bi[j];
        bd[j] = lt ? d : od;
        bi[j] = lt ? id : oi;
        d = lt ? od : d;
        id = lt ? oi : id;
    }
}

// ---------------------------------------------------------------- wave64
__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }
// number of set bits of m below the calling lane
__device__ __forceinline__ uint32_t count_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    uint32_t lo = shfl_u32((uint32_t)v, src), hi = shfl_u32((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    for (int o = 32; o >= 1; o >>= 1) v = min(v, shfl_u32(v, (int)(lane_id() ^ o)));
    return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    for (int o = 32; o >= 1; o >>= 1) v = max(v, shfl_u32(v, (int)(lane_id() ^ o)));
    return v;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int o = 32; o >= 1; o >>= 1) v += shfl_u32(v, (int)(lane_id() ^ o));
    return v;
}

// Inclusive scan of one value per thread over a 256-thread block (all
// threads must call it; s_wsum holds 4 words of LDS).
__device__ __forceinline__ uint32_t block_incl_scan256(uint32_t v, uint32_t* s_wsum) {
    const uint32_t lane = lane_id();
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = shfl_u32(v, (int)lane - o);
        if (lane >= (uint32_t)o) v += t;
    }
    if (lane == 63) s_wsum[w] = v;
    __syncthreads();
    uint32_t add = 0;
    for (int i = 0; i < w; ++i) add += s_wsum[i];
    __syncthreads();
    return v + add;
}

}  // namespace psi
