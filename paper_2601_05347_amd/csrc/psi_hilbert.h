// Table-driven Hilbert keys for the kernels (build encode, leaf fill, updates, queries).
//
// The Hilbert key of Sec. 2.2 (Skilling's construction, as computed by
// hilbert_key in psi_dev.h) reads the point plane by plane from the top.
// Every plane's work depends on the bits of that plane and on a small state:
// the exchanges and reflections applied so far to the lower planes (a signed
// permutation of the axes) plus the parity that the Gray-code step carries
// down from the planes above. Walking that finite-state machine over the
// point's bit planes, several planes per table lookup, gives the same key
// with a fraction of the ALU work; the inverse machine walks a key back to
// the point. A lookup's chunk holds the P plane bits of each axis side by
// side (axis d at bits [d P, d P + P)), so both directions take them from and
// give them to the coordinates with one bit-field operation per axis.
//
// The tables are generated at compile time from the plane rule itself:
//  * current bits  c_d = o[perm[d]] ^ flip_d   (o: the point's bits in the plane)
//  * Gray code     g_d = c_0 ^ ... ^ c_d, key bits g_d ^ par (axis 0 first)
//  * next parity   par ^ g_{D-1}
//  * then for d = 0 .. D-1: c_d set -> reflect axis 0, else exchange axes 0, d.
// 2D: 8 reachable states, 4 planes per lookup (32 planes: 8 lookups).
// 3D: 48 reachable states, the top plane alone, then 2 planes per lookup
// (21 planes: 1 + 10 lookups).
#pragma once
#include <stdint.h>

#include "psi_dev.h"

namespace psi {

template <int D> struct HilbertFsm {
    static constexpr int W = KeyBits<D>::W;        // planes
    static constexpr int P = D == 2 ? 4 : 2;       // planes per main lookup
    static constexpr int TOP = D == 2 ? 0 : 1;     // planes of the first, single-plane step
    static constexpr int STEPS = (W - TOP) / P;    // main lookups
    static constexpr int CH = 1 << (D * P);        // chunk values
    static constexpr int S = D == 2 ? 8 : 48;      // reachable states
    static constexpr int MAIN = S * CH;
    static constexpr int ENTRIES = MAIN + (TOP ? (1 << D) : 0);
    static_assert(TOP + STEPS * P == W, "planes must split into the lookups");
    // entry = (next state << 8) | output chunk; enc maps an axis-grouped
    // chunk -> key chunk, dec maps key chunk -> axis-grouped chunk. The
    // single-plane entries of the top step (from state 0) follow the main
    // table (one bit per axis, axis d at bit d).
    uint16_t enc[ENTRIES];
    uint16_t dec[ENTRIES];
};

namespace fsm_detail {

struct St {
    int perm[3];
    int flip;
    int par;
};

// One plane: o holds the point's bit of axis d at bit d (Morton order);
// returns the key's D bits for the plane, axis 0 most significant.
constexpr int plane(St& st, int o, int D) {
    int c[3] = {0, 0, 0};
    for (int d = 0; d < D; ++d) c[d] = ((o >> st.perm[d]) & 1) ^ ((st.flip >> d) & 1);
    int out = 0, acc = 0;
    for (int d = 0; d < D; ++d) {
        acc ^= c[d];
        out |= (acc ^ st.par) << (D - 1 - d);
    }
    st.par ^= acc;
    for (int d = 0; d < D; ++d) {
        if (c[d]) {
            st.flip ^= 1;
        } else if (d) {
            const int tp = st.perm[0];
            st.perm[0] = st.perm[d];
            st.perm[d] = tp;
            const int f0 = st.flip & 1, fd = (st.flip >> d) & 1;
            st.flip = (st.flip & ~1 & ~(1 << d)) | fd | (f0 << d);
        }
    }
    return out;
}

constexpr int code(const St& x) { return ((x.perm[0] + 3 * x.perm[1] + 9 * x.perm[2]) * 8 + x.flip) * 2 + x.par; }

// Plane-major chunk (plane j's axis bits at [D j, D j + D), axis d at bit d of
// its plane) -> axis-grouped chunk (axis d's plane bits at [d P, d P + P),
// plane j at bit j).
constexpr int grouped(int ch, int D, int P) {
    int g = 0;
    for (int j = 0; j < P; ++j)
        for (int d = 0; d < D; ++d) g |= ((ch >> (D * j + d)) & 1) << (d * P + j);
    return g;
}
constexpr int CODES = 27 * 8 * 2;

template <int D> constexpr HilbertFsm<D> make() {
    using F = HilbertFsm<D>;
    HilbertFsm<D> t{};
    St list[F::S] = {};
    int idx[CODES] = {};
    for (int c = 0; c < CODES; ++c) idx[c] = -1;
    for (int d = 0; d < 3; ++d) list[0].perm[d] = d;
    idx[code(list[0])] = 0;
    int n = 1;
    for (int i = 0; i < n; ++i) {
        for (int v = 0; v < (1 << D); ++v) {
            St x = list[i];
            plane(x, v, D);
            if (idx[code(x)] < 0 && n < F::S) {
                idx[code(x)] = n;
                list[n++] = x;
            }
        }
    }
    for (int s = 0; s < F::S; ++s) {
        for (int ch = 0; ch < F::CH; ++ch) {
            St x = list[s];
            int out = 0;
            for (int j = F::P - 1; j >= 0; --j) out = (out << D) | plane(x, (ch >> (D * j)) & ((1 << D) - 1), D);
            const int nx = idx[code(x)];
            const int g = grouped(ch, D, F::P);
            t.enc[s * F::CH + g] = (uint16_t)((nx << 8) | out);
            t.dec[s * F::CH + out] = (uint16_t)((nx << 8) | g);
        }
    }
    if (F::TOP) {
        for (int v = 0; v < (1 << D); ++v) {
            St x = list[0];
            const int out = plane(x, v, D);
            const int nx = idx[code(x)];
            t.enc[F::MAIN + v] = (uint16_t)((nx << 8) | out);
            t.dec[F::MAIN + out] = (uint16_t)((nx << 8) | v);
        }
    }
    return t;
}

}  // namespace fsm_detail

// Device copies (constant memory); kernels stage the one they use in LDS.
__constant__ const HilbertFsm<2> kHilbert2 = fsm_detail::make<2>();
__constant__ const HilbertFsm<3> kHilbert3 = fsm_detail::make<3>();

template <int D> __device__ __forceinline__ const HilbertFsm<D>& hilbert_fsm() {
    if constexpr (D == 2) return kHilbert2;
    else return kHilbert3;
}

// Copies the encode (enc = true) or decode table into LDS; all threads of the
// block call it, followed by a barrier of the caller's.
template <int D>
__device__ __forceinline__ void stage_hilbert(uint16_t* s_tab, bool enc) {
    using F = HilbertFsm<D>;
    const uint16_t* src = enc ? hilbert_fsm<D>().enc : hilbert_fsm<D>().dec;
    for (int i = threadIdx.x; i < F::ENTRIES; i += blockDim.x) s_tab[i] = src[i];
}

template <int D> __device__ __forceinline__ uint64_t hilbert_key_fsm(const uint32_t* p, const uint16_t* s_enc) {
    using F = HilbertFsm<D>;
    uint32_t st = 0;
    uint64_t k = 0;
    if constexpr (F::TOP == 1) {
        uint32_t v = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) v |= ((p[d] >> (F::W - 1)) & 1u) << d;
        const uint32_t e = s_enc[F::MAIN + v];
        k = e & 0xFFu;
        st = e >> 8;
    }
#pragma unroll
    for (int c = F::STEPS - 1; c >= 0; --c) {
        uint32_t ch = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) ch |= ((p[d] >> (F::P * c)) & ((1u << F::P) - 1u)) << (d * F::P);
        const uint32_t e = s_enc[st * F::CH + ch];
        k = (k << (D * F::P)) | (e & 0xFFu);
        st = e >> 8;
    }
    return k;
}

template <int D> __device__ __forceinline__ void hilbert_point_fsm(uint64_t k, uint32_t* p, const uint16_t* s_dec) {
    using F = HilbertFsm<D>;
    uint32_t st = 0;
    uint32_t x[D];
#pragma unroll
    for (int d = 0; d < D; ++d) x[d] = 0;
    if constexpr (F::TOP == 1) {
        const uint32_t e = s_dec[F::MAIN + (uint32_t)(k >> (D * (F::W - 1)))];
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = (e >> d) & 1u;
        st = e >> 8;
    }
#pragma unroll
    for (int c = F::STEPS - 1; c >= 0; --c) {
        const uint32_t ch = (uint32_t)(k >> (D * F::P * c)) & (F::CH - 1);
        const uint32_t e = s_dec[st * F::CH + ch];
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = (x[d] << F::P) | ((e >> (d * F::P)) & ((1u << F::P) - 1u));
        st = e >> 8;
    }
#pragma unroll
    for (int d = 0; d < D; ++d) p[d] = x[d];
}

// Curve keys and points through the tables read straight from constant
// memory (for kernels that code a few keys per thread and do not stage the
// tables); Morton keys need no table.
template <int D, int CURVE> __device__ __forceinline__ uint64_t sfc_key_tab(const uint32_t* p) {
    if constexpr (CURVE == 0) return morton_key<D>(p);
    else return hilbert_key_fsm<D>(p, hilbert_fsm<D>().enc);
}
template <int D, int CURVE> __device__ __forceinline__ void sfc_point_tab(uint64_t k, uint32_t* p) {
    if constexpr (CURVE == 0) morton_point<D>(k, p);
    else hilbert_point_fsm<D>(k, p, hilbert_fsm<D>().dec);
}

}  // namespace psi
