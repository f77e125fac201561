// Two-level sort of a build's (key, id) pairs.
//
// The build sort of Alg. 3 is a sample sort: distribute the (code, id) pairs
// into buckets, then sort every bucket on its own, where it fits in cache.
// The same shape here, with radix digits in place of sampled pivots: two
// global LSD passes order the pairs by their top 16 key bits (65536
// buckets), then every bucket of at most BUCKET_MAX pairs is sorted entirely
// inside one workgroup's LDS, in place: one counting pass into 256
// sub-buckets, then one thread sorts each sub-bucket in registers. Buckets
// of up to BUCKET_HUGE pairs take a 1024-thread variant of the same scheme;
// larger ones (clustered data) are sorted by six segmented global passes
// instead. Traffic for uniform data: two global passes plus one read and one
// write of every pair, instead of eight global passes.
#include "psi_kern.h"

namespace psi {

namespace {

inline unsigned blocks_for(uint64_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }


// bstart[t] = first position whose top bits (key >> shift) are >= t, for
// t in [0, nb]; the keys are already ordered by those bits.
__global__ void k_bucket_starts(const uint64_t* __restrict__ keys, uint64_t n, const uint32_t* __restrict__ top,
                                uint32_t nb, uint32_t* __restrict__ bstart) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > nb) return;
    const uint32_t shift = *top;
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if ((keys[mid] >> shift) < t) lo = mid + 1;
        else hi = mid;
    }
    bstart[t] = (uint32_t)lo;
}

// Ascending bitonic network over N (key, id) pairs held in registers; pairs
// compare lexicographically (ids are unique, so the order is total).
template <int N>
__device__ __forceinline__ void bitonic(uint64_t (&k)[N], uint32_t (&id)[N]) {
#pragma unroll
    for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ stride;
                if (l > i) {
                    const bool up = (i & size) == 0;
                    const bool gt = k[i] > k[l] || (k[i] == k[l] && id[i] > id[l]);
                    if (gt == up) {
                        const uint64_t tk = k[i];
                        k[i] = k[l];
                        k[l] = tk;
                        const uint32_t ti = id[i];
                        id[i] = id[l];
                        id[l] = ti;
                    }
                }
            }
        }
    }
}

// Sorts the run s_k/s_i[s0, s0 + c) (c <= N) in place, in registers.
template <int N>
__device__ __forceinline__ void sort_run(uint64_t* s_k, uint32_t* s_i, uint32_t s0, uint32_t c) {
    uint64_t k[N];
    uint32_t id[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const bool ok = (uint32_t)j < c;
        k[j] = ok ? s_k[s0 + j] : ~0ull;
        id[j] = ok ? s_i[s0 + j] : ~0u;
    }
    bitonic<N>(k, id);
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if ((uint32_t)j < c) {
            s_k[s0 + j] = k[j];
            s_i[s0 + j] = id[j];
        }
    }
}

constexpr uint32_t RUN_NET = 16;  // largest sub-bucket one thread sorts with a network
constexpr uint32_t RUN_WAVE = 64;  // largest sub-bucket a wave sorts by ranking

// A wave sorts the sub-buckets of its lanes that hold more than RUN_NET pairs
// (and at most RUN_WAVE), one after the other: lane x takes pair x and counts
// the pairs of the sub-bucket that precede it.
__device__ __forceinline__ void rank_runs(uint64_t* s_k, uint32_t* s_i, uint32_t s0, uint32_t c) {
    const uint32_t lane = lane_id();
    uint64_t todo = ballot(c > RUN_NET);
    while (todo) {
        const int src = __builtin_ctzll(todo);
        todo &= todo - 1;
        const uint32_t rs = shfl_u32(s0, src), rc = shfl_u32(c, src);
        const bool on = lane < rc;
        const uint64_t mk = on ? s_k[rs + lane] : ~0ull;
        const uint32_t mi = on ? s_i[rs + lane] : ~0u;
        uint32_t rank = 0;
        for (uint32_t x = 0; x < rc; ++x) {  // same trip count on every lane: all reads precede the writes
            const uint64_t ok = s_k[rs + x];
            const uint32_t oi = s_i[rs + x];
            rank += (ok < mk || (ok == mk && oi < mi)) ? 1u : 0u;
        }
        if (on) {
            s_k[rs + rank] = mk;
            s_i[rs + rank] = mi;
        }
    }
}

// One workgroup per bucket of at most BMAX pairs, sorted in place by (key,
// id). The BUCKET_SMALL variant runs first over all buckets and flags the
// larger ones; the BUCKET_MAX variant then takes those of at most BUCKET_MAX
// pairs (half the occupancy, for the rare large buckets). The pairs arrive in
// id order (the global passes are stable).
// Sub-buckets: the 8 key bits just below the highest bit in which the
// bucket's keys differ (so that clustered buckets still spread); a thread
// sorts its sub-bucket in registers (at most RUN_NET pairs), a wave ranks the
// larger ones (at most RUN_WAVE). A bucket with a larger sub-bucket (skewed)
// is sorted by the BUCKET_MAX variant instead, by stable 8-bit LSD passes
// over the bits [0, lo_bits) in LDS: the BUCKET_SMALL variant flags it
// (big[t] = 2) and leaves its pairs alone. Buckets above BMAX are only
// flagged (big[t] = 1). Decreasing bucket starts (pairs not ordered by their
// top bits) latch ERR_SPIN and the bucket is left alone.
template <int BMAX>
__global__ __launch_bounds__(256) void k_local_sort(uint64_t* __restrict__ keys, uint32_t* __restrict__ ids,
                                                    const uint32_t* __restrict__ bstart,
                                                    const uint32_t* __restrict__ top, uint32_t* __restrict__ big,
                                                    uint32_t* __restrict__ err) {
    const uint32_t lo_bits = *top;
    constexpr int IPT = BMAX / 256;  // items per thread at the largest bucket
    // the light variant has no LSD path (it leaves skewed buckets to the wide
    // one): fewer registers and less LDS, six workgroups per CU
    constexpr bool LSD = BMAX != BUCKET_SMALL;
    __shared__ uint64_t s_k[BMAX];
    __shared__ uint32_t s_i[BMAX];
    __shared__ uint32_t s_cnt[LSD ? 4 : 2][RADIX];
    __shared__ uint32_t s_wsum[4];
    __shared__ uint64_t s_red[8];
    __shared__ uint32_t s_wmax[4];
    __shared__ uint32_t s_skip[LSD ? 8 : 1];  // one flag per LSD pass: no reset races between passes
    const uint32_t t = blockIdx.x;
    const uint32_t b = bstart[t], e = bstart[t + 1];
    if (e < b) {
        if (threadIdx.x == 0) {
            big[t] = 0u;
            atomicOr(err, ERR_SPIN);
        }
        return;
    }
    const uint32_t size = e - b;
    if (BMAX == BUCKET_SMALL) {  // first launch: every bucket gets its flag
        if (threadIdx.x == 0) big[t] = size > (uint32_t)BMAX ? 1u : 0u;
        if (size <= 1 || size > (uint32_t)BMAX) return;
    } else {  // second launch: only the buckets the first one left (larger, or skewed)
        if (size > (uint32_t)BMAX || (size <= (uint32_t)BUCKET_SMALL && big[t] != 2u)) return;
        __syncthreads();  // every thread has read the flag
        if (threadIdx.x == 0) big[t] = 0u;
    }
    const int w = threadIdx.x >> 6;
    const uint32_t lane = lane_id();
    // wave w owns positions [w*chunk, (w+1)*chunk): all four waves stay busy
    // and item order (wave, item, lane) is position order
    const uint32_t chunk = ((size + 3) / 4 + 63) & ~63u;
    const uint32_t nit = chunk / 64;
    uint64_t k[IPT];
    uint32_t id[IPT];
    uint32_t rk[IPT];
    uint64_t mn = ~0ull, mx = 0;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const uint32_t pos = w * chunk + i * 64 + lane;
        const bool ok = (uint32_t)i < nit && pos < size;
        k[i] = ok ? keys[b + pos] : 0ull;
        id[i] = ok ? ids[b + pos] : 0u;
        if (ok) {
            mn = min(mn, k[i]);
            mx = max(mx, k[i]);
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        mn = min(mn, shfl_u64(mn, (int)(lane ^ o)));
        mx = max(mx, shfl_u64(mx, (int)(lane ^ o)));
    }
    for (int x = threadIdx.x; x < RADIX; x += 256) s_cnt[0][x] = 0;
    if (LSD && threadIdx.x < 8) s_skip[threadIdx.x] = 0;
    if (lane == 0) {
        s_red[w] = mn;
        s_red[4 + w] = mx;
    }
    __syncthreads();
    mn = min(min(s_red[0], s_red[1]), min(s_red[2], s_red[3]));
    mx = max(max(s_red[4], s_red[5]), max(s_red[6], s_red[7]));
    if (mn == mx) return;  // one key: already in id order
    const int hb = 63 - __clzll(mn ^ mx);
    const uint32_t sh = hb >= 7 ? (uint32_t)hb - 7 : 0u;
    // sub-bucket counts; the slot inside a sub-bucket is arbitrary (the
    // sub-bucket sort orders it)
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        if ((uint32_t)i >= nit) break;
        const uint32_t pos = w * chunk + i * 64 + lane;
        if (pos < size) rk[i] = atomicAdd(&s_cnt[0][(uint32_t)(k[i] >> sh) & (RADIX - 1)], 1u);
    }
    __syncthreads();
    const uint32_t c = s_cnt[0][threadIdx.x];
    const uint32_t s0 = block_incl_scan256(c, s_wsum) - c;
    const uint32_t wm = wave_max_u32(c);  // all lanes take part in the shuffles
    s_cnt[1][threadIdx.x] = s0;
    if (lane == 0) s_wmax[w] = wm;
    __syncthreads();
    const uint32_t bm = max(max(s_wmax[0], s_wmax[1]), max(s_wmax[2], s_wmax[3]));
    if (bm <= RUN_WAVE) {
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if ((uint32_t)i >= nit) break;
            const uint32_t pos = w * chunk + i * 64 + lane;
            if (pos < size) {
                const uint32_t lp = s_cnt[1][(uint32_t)(k[i] >> sh) & (RADIX - 1)] + rk[i];
                s_k[lp] = k[i];
                s_i[lp] = id[i];
            }
        }
        __syncthreads();
        const uint32_t cn = c <= RUN_NET ? c : 0u;
        const uint32_t wn = wave_max_u32(cn);  // uniform over the wave
        if (wn <= 8) sort_run<8>(s_k, s_i, s0, cn);
        else sort_run<16>(s_k, s_i, s0, cn);
        rank_runs(s_k, s_i, s0, c);
        __syncthreads();
        for (uint32_t pos = threadIdx.x; pos < size; pos += 256) {
            keys[b + pos] = s_k[pos];
            ids[b + pos] = s_i[pos];
        }
        return;
    }
    if constexpr (!LSD) {  // skewed: flagged for the wide variant, pairs untouched
        if (threadIdx.x == 0) big[t] = 2u;
        return;
    } else {
    // skewed bucket: stable LSD passes in LDS
    for (uint32_t shift = 0, pass = 0; shift < lo_bits; shift += RADIX_BITS, ++pass) {
        for (int x = threadIdx.x; x < 4 * RADIX; x += 256) (&s_cnt[0][0])[x] = 0;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if ((uint32_t)i >= nit) break;
            const uint32_t pos = w * chunk + i * 64 + lane;
            const bool ok = pos < size;
            const uint32_t dg = (uint32_t)(k[i] >> shift) & (RADIX - 1);
            uint64_t peers = ballot(ok);
#pragma unroll
            for (int bb = 0; bb < RADIX_BITS; ++bb) {
                const bool bit = (dg >> bb) & 1u;
                const uint64_t m = ballot(bit);
                peers &= bit ? m : ~m;
            }
            const uint32_t below = count_below(peers);
            const uint32_t base = s_cnt[w][dg];
            if (ok && below == 0) s_cnt[w][dg] = base + (uint32_t)__popcll(peers);
            rk[i] = base + below;
        }
        __syncthreads();
        const uint32_t d = threadIdx.x;
        uint32_t tot = 0;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const uint32_t cc = s_cnt[x][d];
            s_cnt[x][d] = tot;
            tot += cc;
        }
        if (tot == size) s_skip[pass] = 1;  // every pair has this digit: the pass changes nothing
        const uint32_t loc = block_incl_scan256(tot, s_wsum) - tot;
#pragma unroll
        for (int x = 0; x < 4; ++x) s_cnt[x][d] += loc;
        __syncthreads();
        if (s_skip[pass]) continue;  // uniform over the block
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if ((uint32_t)i >= nit) break;
            const uint32_t pos = w * chunk + i * 64 + lane;
            if (pos < size) {
                const uint32_t dg = (uint32_t)(k[i] >> shift) & (RADIX - 1);
                const uint32_t lp = s_cnt[w][dg] + rk[i];
                s_k[lp] = k[i];
                s_i[lp] = id[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if ((uint32_t)i >= nit) break;
            const uint32_t pos = w * chunk + i * 64 + lane;
            if (pos < size) {
                k[i] = s_k[pos];
                id[i] = s_i[pos];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        if ((uint32_t)i >= nit) break;
        const uint32_t pos = w * chunk + i * 64 + lane;
        if (pos < size) {
            keys[b + pos] = k[i];
            ids[b + pos] = id[i];
        }
    }
    }
}

// Buckets of BUCKET_MAX + 1 .. BUCKET_HUGE pairs (clustered data, or about
// 7600 pairs per bucket at 5e8 points): the light variant's scheme with four
// times the threads, one sub-bucket per thread (the 10 key bits below the
// highest bit in which the bucket's keys differ) and the bucket staged in
// 96 KB of LDS. One workgroup per CU: workgroup g owns buckets g, g + grid,
// g + 2 grid, ... (at most HUGE_THREADS of them), finds those in range with
// one load per thread, then sorts them one after the other. A bucket with a
// sub-bucket of more than RUN_WAVE pairs is left as it is, flagged, for the
// segmented passes.
constexpr int HUGE_THREADS = 1024;
constexpr int HUGE_WAVES = HUGE_THREADS / 64;
constexpr uint32_t HUGE_SUB = HUGE_THREADS;  // sub-buckets
static_assert(BUCKET_HUGE % HUGE_THREADS == 0, "items per thread");

__global__ __launch_bounds__(HUGE_THREADS) void k_local_sort_huge(uint64_t* __restrict__ keys,
                                                                  uint32_t* __restrict__ ids,
                                                                  const uint32_t* __restrict__ bstart,
                                                                  uint32_t nb, uint32_t* __restrict__ big) {
    constexpr int IPT = BUCKET_HUGE / HUGE_THREADS;
    __shared__ uint64_t s_k[BUCKET_HUGE];
    __shared__ uint32_t s_i[BUCKET_HUGE];
    __shared__ uint32_t s_cnt[HUGE_SUB];
    __shared__ uint32_t s_off[HUGE_SUB];
    __shared__ uint32_t s_wsum[HUGE_WAVES];
    __shared__ uint32_t s_wmax[HUGE_WAVES];
    __shared__ uint64_t s_red[2 * HUGE_WAVES];
    __shared__ uint32_t s_list[HUGE_THREADS];
    __shared__ uint32_t s_nl;
    const int w = threadIdx.x >> 6;
    const uint32_t lane = lane_id();
    if (threadIdx.x == 0) s_nl = 0;
    __syncthreads();
    {
        const uint64_t t = blockIdx.x + (uint64_t)gridDim.x * threadIdx.x;
        if (t < nb) {
            const uint32_t b = bstart[t], e = bstart[t + 1];
            if (e >= b && e - b > (uint32_t)BUCKET_MAX && e - b <= (uint32_t)BUCKET_HUGE)
                s_list[atomicAdd(&s_nl, 1u)] = (uint32_t)t;
        }
    }
    __syncthreads();
    const uint32_t total = s_nl;
    for (uint32_t j = 0; j < total; ++j) {
        __syncthreads();  // the previous bucket's LDS reads are done
        const uint32_t t = s_list[j];
        const uint32_t b = bstart[t], size = bstart[t + 1] - b;
        // wave w owns positions [w*chunk, (w+1)*chunk): item order (wave,
        // item, lane) is position order
        const uint32_t chunk = ((size + HUGE_WAVES - 1) / HUGE_WAVES + 63) & ~63u;
        const uint32_t nit = chunk / 64;
        uint64_t k[IPT];
        uint32_t id[IPT];
        uint32_t rk[IPT];
        uint64_t mn = ~0ull, mx = 0;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const uint32_t pos = w * chunk + i * 64 + lane;
            const bool ok = (uint32_t)i < nit && pos < size;
            k[i] = ok ? keys[b + pos] : 0ull;
            id[i] = ok ? ids[b + pos] : 0u;
            if (ok) {
                mn = min(mn, k[i]);
                mx = max(mx, k[i]);
            }
        }
        for (int o = 32; o >= 1; o >>= 1) {
            mn = min(mn, shfl_u64(mn, (int)(lane ^ o)));
            mx = max(mx, shfl_u64(mx, (int)(lane ^ o)));
        }
        s_cnt[threadIdx.x] = 0;
        if (lane == 0) {
            s_red[w] = mn;
            s_red[HUGE_WAVES + w] = mx;
        }
        __syncthreads();
        mn = s_red[0];
        mx = s_red[HUGE_WAVES];
#pragma unroll
        for (int x = 1; x < HUGE_WAVES; ++x) {
            mn = min(mn, s_red[x]);
            mx = max(mx, s_red[HUGE_WAVES + x]);
        }
        if (mn == mx) {  // one key: already in id order
            if (threadIdx.x == 0) big[t] = 0u;
            continue;
        }
        const int hb = 63 - __clzll(mn ^ mx);
        const uint32_t sh = hb >= 9 ? (uint32_t)hb - 9 : 0u;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if ((uint32_t)i >= nit) break;
            const uint32_t pos = w * chunk + i * 64 + lane;
            if (pos < size) rk[i] = atomicAdd(&s_cnt[(uint32_t)(k[i] >> sh) & (HUGE_SUB - 1)], 1u);
        }
        __syncthreads();
        const uint32_t c = s_cnt[threadIdx.x];
        const uint32_t s0 = block_incl_scan256(c, s_wsum) - c;
        const uint32_t wm = wave_max_u32(c);
        s_off[threadIdx.x] = s0;
        if (lane == 0) s_wmax[w] = wm;
        __syncthreads();
        uint32_t bm = s_wmax[0];
#pragma unroll
        for (int x = 1; x < HUGE_WAVES; ++x) bm = max(bm, s_wmax[x]);
        if (bm > RUN_WAVE) continue;  // skewed: the segmented passes take it
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if ((uint32_t)i >= nit) break;
            const uint32_t pos = w * chunk + i * 64 + lane;
            if (pos < size) {
                const uint32_t lp = s_off[(uint32_t)(k[i] >> sh) & (HUGE_SUB - 1)] + rk[i];
                s_k[lp] = k[i];
                s_i[lp] = id[i];
            }
        }
        __syncthreads();
        const uint32_t cn = c <= RUN_NET ? c : 0u;
        const uint32_t wn = wave_max_u32(cn);  // uniform over the wave
        if (wn <= 8) sort_run<8>(s_k, s_i, s0, cn);
        else sort_run<16>(s_k, s_i, s0, cn);
        rank_runs(s_k, s_i, s0, c);
        __syncthreads();
        for (uint32_t pos = threadIdx.x; pos < size; pos += HUGE_THREADS) {
            keys[b + pos] = s_k[pos];
            ids[b + pos] = s_i[pos];
        }
        if (threadIdx.x == 0) big[t] = 0u;
    }
}

// Histograms of the two bucket digits (bits [s0, s0 + 8) and [s1, s1 + 8))
// of every key; eight loads in flight per thread.
__global__ __launch_bounds__(256) void k_hist_keys2(const uint64_t* __restrict__ keys, uint64_t n, uint32_t s0,
                                                    uint32_t s1, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[2][RADIX];
    for (int i = threadIdx.x; i < 2 * RADIX; i += blockDim.x) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 7 * stride < n; i += 8 * stride) {
        uint64_t k[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) k[j] = keys[i + j * stride];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            atomicAdd(&h[0][(uint32_t)(k[j] >> s0) & (RADIX - 1)], 1u);
            atomicAdd(&h[1][(uint32_t)(k[j] >> s1) & (RADIX - 1)], 1u);
        }
    }
    for (; i < n; i += stride) {
        const uint64_t k = keys[i];
        atomicAdd(&h[0][(uint32_t)(k >> s0) & (RADIX - 1)], 1u);
        atomicAdd(&h[1][(uint32_t)(k >> s1) & (RADIX - 1)], 1u);
    }
    __syncthreads();
    for (int x = threadIdx.x; x < 2 * RADIX; x += blockDim.x) {
        const uint32_t v = (&h[0][0])[x];
        if (v) atomicAdd(&hist[x], v);
    }
}

// Counts for the two chunked bucket passes (bits [s0, s0 + 8) = d0 and
// [s1, s1 + 8) = d1 of every key): cnt[0][x][d0] over the keys of input chunk
// x (tiles T x / 8 .. T (x + 1) / 8), cnt[1][g][d1] over the keys whose d0
// lies in [32 g, 32 g + 32) (the g-th group of the first pass's output).
// Each workgroup reads one contiguous range, eight loads in flight per thread.
// With `redo` set (device word), the kernel counts only if *redo is nonzero,
// and the digits sit at bits *top and *top + 8 instead.
__global__ __launch_bounds__(256) void k_hist_chunks(const uint64_t* __restrict__ keys, uint64_t n, uint32_t s0,
                                                     uint32_t s1, uint64_t T, uint32_t* __restrict__ cnt,
                                                     const uint32_t* __restrict__ redo,
                                                     const uint32_t* __restrict__ top) {
    if (redo) {
        if (*redo == 0) return;
        s0 = *top;
        s1 = s0 + 8;
    }
    __shared__ uint32_t h[2][XCD_CHUNKS][RADIX];
    for (int i = threadIdx.x; i < 2 * (int)XCD_CHUNKS * RADIX; i += blockDim.x) (&h[0][0][0])[i] = 0;
    __syncthreads();
    uint64_t bnd[XCD_CHUNKS];  // first tile of chunks 1 .. 7 (bnd[0] unused)
#pragma unroll
    for (uint32_t x = 0; x < XCD_CHUNKS; ++x) bnd[x] = T * x / XCD_CHUNKS;
    const uint64_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t b = (uint64_t)blockIdx.x * per, e = min<uint64_t>(b + per, n);
    auto count = [&](uint64_t i, uint64_t k) {
        const uint64_t t = i / SORT_TILE;
        uint32_t x = 0;
#pragma unroll
        for (uint32_t y = 1; y < XCD_CHUNKS; ++y) x += t >= bnd[y] ? 1u : 0u;
        const uint32_t d0 = (uint32_t)(k >> s0) & (RADIX - 1), d1 = (uint32_t)(k >> s1) & (RADIX - 1);
        atomicAdd(&h[0][x][d0], 1u);
        atomicAdd(&h[1][d0 >> 5][d1], 1u);
    };
    uint64_t i = b + threadIdx.x;
    for (; i + 7 * blockDim.x < e; i += 8 * blockDim.x) {
        uint64_t k[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) k[j] = keys[i + j * blockDim.x];
#pragma unroll
        for (int j = 0; j < 8; ++j) count(i + j * blockDim.x, k[j]);
    }
    for (; i < e; i += blockDim.x) count(i, keys[i]);
    __syncthreads();
    for (int x = threadIdx.x; x < 2 * (int)XCD_CHUNKS * RADIX; x += blockDim.x) {
        const uint32_t v = (&h[0][0][0])[x];
        if (v) atomicAdd(&cnt[x], v);
    }
}

// From those counts (one workgroup of 256 threads): the digit offsets of
// every chunk of both passes and the chunk tables (tb1 / tb2: first tile,
// tiles, first position, end position; XCD_CHUNKS entries each).
__global__ __launch_bounds__(256) void k_chunk_offsets(const uint32_t* __restrict__ cnt, uint64_t n, uint64_t T,
                                                       uint32_t* __restrict__ off1, uint32_t* __restrict__ off2,
                                                       uint32_t* __restrict__ tb1_first, uint32_t* __restrict__ tb1_nt,
                                                       uint64_t* __restrict__ tb1_b, uint64_t* __restrict__ tb1_e,
                                                       uint32_t* __restrict__ tb2_first, uint32_t* __restrict__ tb2_nt,
                                                       uint64_t* __restrict__ tb2_b, uint64_t* __restrict__ tb2_e) {
    __shared__ uint32_t s_wsum[4];
    __shared__ uint32_t s_g0[RADIX];
    __shared__ uint32_t s_nt[XCD_CHUNKS];
    const uint32_t d = threadIdx.x;
    const uint32_t* c1 = cnt;
    const uint32_t* c2 = cnt + XCD_CHUNKS * RADIX;
    uint32_t t0 = 0, t1 = 0;
    for (uint32_t x = 0; x < XCD_CHUNKS; ++x) {
        t0 += c1[x * RADIX + d];
        t1 += c2[x * RADIX + d];
    }
    const uint32_t g0 = block_incl_scan256(t0, s_wsum) - t0;
    const uint32_t g1 = block_incl_scan256(t1, s_wsum) - t1;
    s_g0[d] = g0;
    uint32_t r0 = g0, r1 = g1;
    for (uint32_t x = 0; x < XCD_CHUNKS; ++x) {
        off1[x * RADIX + d] = r0;
        r0 += c1[x * RADIX + d];
        off2[x * RADIX + d] = r1;
        r1 += c2[x * RADIX + d];
    }
    __syncthreads();
    if (d < XCD_CHUNKS) {
        const uint64_t fb = T * d / XCD_CHUNKS, fe = T * (d + 1) / XCD_CHUNKS;
        tb1_first[d] = (uint32_t)fb;
        tb1_nt[d] = (uint32_t)(fe - fb);
        tb1_b[d] = min<uint64_t>(fb * SORT_TILE, n);
        tb1_e[d] = min<uint64_t>(fe * SORT_TILE, n);
        const uint64_t sb = s_g0[32 * d], se = d + 1 < XCD_CHUNKS ? s_g0[32 * (d + 1)] : n;
        const uint32_t nt = (uint32_t)((se - sb + SORT_TILE - 1) / SORT_TILE);
        s_nt[d] = nt;
        tb2_nt[d] = nt;
        tb2_b[d] = sb;
        tb2_e[d] = se;
    }
    __syncthreads();
    if (d < XCD_CHUNKS) {
        uint32_t f = 0;
        for (uint32_t x = 0; x < d; ++x) f += s_nt[x];
        tb2_first[d] = f;
    }
}

__global__ void k_big_count(const uint32_t* __restrict__ bstart, const uint32_t* __restrict__ big, uint32_t nb,
                            uint32_t* __restrict__ ntiles) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb) return;
    ntiles[t] = big[t] ? (bstart[t + 1] - bstart[t] + SORT_TILE - 1) / SORT_TILE : 0u;
}

// Segment tables of the big buckets (segment s = the s-th big bucket).
__global__ void k_big_tables(const uint32_t* __restrict__ bstart, const uint32_t* __restrict__ big,
                             const uint32_t* __restrict__ big_idx, const uint32_t* __restrict__ tile_off,
                             uint32_t nb, uint32_t* __restrict__ tile_seg, uint32_t* __restrict__ tile_beg,
                             uint32_t* __restrict__ seg_first, uint32_t* __restrict__ seg_end,
                             uint64_t* __restrict__ seg_begin) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb || !big[t]) return;
    const uint32_t s = big_idx[t];
    const uint32_t b = bstart[t], e = bstart[t + 1];
    seg_first[s] = tile_off[t];
    seg_end[s] = e;
    seg_begin[s] = b;
    uint32_t j = tile_off[t];
    for (uint32_t p = b; p < e; p += SORT_TILE, ++j) {
        tile_seg[j] = s;
        tile_beg[j] = p;
    }
}

// Per-segment histograms of the low six digits, tile by tile (the block
// takes tiles blockIdx.x, + gridDim.x, ... below *ntiles).
__global__ __launch_bounds__(256) void k_seg_hist_keys(const uint64_t* __restrict__ keys, SegTiles sg,
                                                       const uint32_t* __restrict__ ntiles,
                                                       uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[6][RADIX];
    const uint32_t nt = *ntiles;
    for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
        __syncthreads();
        for (int i = threadIdx.x; i < 6 * RADIX; i += blockDim.x) (&h[0][0])[i] = 0;
        __syncthreads();
        const uint32_t s = sg.tile_seg[tile];
        const uint64_t beg = sg.tile_beg[tile];
        const uint64_t end = min<uint64_t>(beg + SORT_TILE, sg.seg_end[s]);
        for (uint64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
            const uint64_t k = keys[i];
#pragma unroll
            for (int p = 0; p < 6; ++p) atomicAdd(&h[p][(k >> (8 * p)) & 255u], 1u);
        }
        __syncthreads();
        uint32_t* hs = hist + (uint64_t)s * 8 * RADIX;
        for (int i = threadIdx.x; i < 6 * RADIX; i += blockDim.x) {
            const uint32_t v = (&h[0][0])[i];
            if (v) atomicAdd(&hs[i], v);
        }
    }
}

// The bucket bits: the 16 below the largest key's leading bit (0 if it has
// at most 16 bits); redo = they differ from the guess the counts were taken
// for while encoding.
__global__ void k_fix_top(const uint64_t* __restrict__ kmax, uint32_t guess, uint32_t* __restrict__ top,
                          uint32_t* __restrict__ redo) {
    if (threadIdx.x | blockIdx.x) return;
    const uint64_t km = *kmax;
    const uint32_t bits = km ? 64u - (uint32_t)__clzll((long long)km) : 0u;
    const uint32_t t = bits > 16 ? bits - 16 : 0u;
    *top = t;
    *redo = t != guess ? 1u : 0u;
}

// p[0 .. words_per * *count) = 0.
__global__ void k_zero_counted(uint32_t* __restrict__ p, uint64_t words_per, const uint32_t* __restrict__ count) {
    const uint64_t n = words_per * *count;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace

void launch_bucket_starts(hipStream_t st, const uint64_t* keys, uint64_t n, const uint32_t* top, uint32_t* bstart,
                          uint32_t nb) {
    hipLaunchKernelGGL(k_bucket_starts, dim3(blocks_for((uint64_t)nb + 1, 256)), dim3(256), 0, st, keys, n, top,
                       nb, bstart);
}

void launch_local_sort(hipStream_t st, uint64_t* keys, uint32_t* ids, const uint32_t* bstart, uint32_t nb,
                       const uint32_t* top, uint32_t* big, uint32_t* err, bool wide) {
    if (wide) hipLaunchKernelGGL(k_local_sort<BUCKET_MAX>, dim3(nb), dim3(256), 0, st, keys, ids, bstart, top, big, err);
    else hipLaunchKernelGGL(k_local_sort<BUCKET_SMALL>, dim3(nb), dim3(256), 0, st, keys, ids, bstart, top, big, err);
}

void launch_local_sort_huge(hipStream_t st, uint64_t* keys, uint32_t* ids, const uint32_t* bstart, uint32_t nb,
                            uint32_t* big) {
    // 256 workgroups (one per CU), more if a workgroup would own more
    // buckets than it has threads
    const uint32_t grid = std::max<uint32_t>(256u, (nb + HUGE_THREADS - 1) / HUGE_THREADS);
    hipLaunchKernelGGL(k_local_sort_huge, dim3(grid), dim3(HUGE_THREADS), 0, st, keys, ids, bstart, nb, big);
}

void launch_fix_top(hipStream_t st, const uint64_t* kmax, uint32_t guess, uint32_t* top, uint32_t* redo) {
    hipLaunchKernelGGL(k_fix_top, dim3(1), dim3(64), 0, st, kmax, guess, top, redo);
}

void launch_zero_counted(hipStream_t st, uint32_t* p, uint64_t words_per, const uint32_t* count, uint64_t max_count) {
    const uint64_t n = words_per * max_count;
    if (!n) return;
    unsigned g = blocks_for(n, 256);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_zero_counted, dim3(g), dim3(256), 0, st, p, words_per, count);
}

void launch_big_tables(hipStream_t st, const uint32_t* bstart, const uint32_t* big, uint32_t nb, uint32_t* ntiles,
                       uint32_t* tile_off, uint32_t* big_idx, uint32_t* totals, uint32_t* tmp) {
    hipLaunchKernelGGL(k_big_count, dim3(blocks_for(nb, 256)), dim3(256), 0, st, bstart, big, nb, ntiles);
    ScanSet ss{};  // both scans in one set of launches
    ss.in[0] = ntiles;
    ss.out[0] = tile_off;
    ss.total[0] = totals;
    ss.n[0] = nb;
    ss.in[1] = big;
    ss.out[1] = big_idx;
    ss.total[1] = totals + 1;
    ss.n[1] = nb;
    launch_scan_multi(st, ss, 2, tmp);
}

void launch_big_fill(hipStream_t st, const uint32_t* bstart, const uint32_t* big, const uint32_t* big_idx,
                     const uint32_t* tile_off, uint32_t nb, const SegTiles& sg, uint64_t* seg_begin) {
    hipLaunchKernelGGL(k_big_tables, dim3(blocks_for(nb, 256)), dim3(256), 0, st, bstart, big, big_idx, tile_off, nb,
                       const_cast<uint32_t*>(sg.tile_seg), const_cast<uint32_t*>(sg.tile_beg),
                       const_cast<uint32_t*>(sg.seg_first_tile), const_cast<uint32_t*>(sg.seg_end), seg_begin);
}

void launch_hist_keys2(hipStream_t st, const uint64_t* keys, uint64_t n, uint32_t s0, uint32_t s1, uint32_t* hist) {
    if (n == 0) return;
    unsigned g = blocks_for(n, 256 * 8);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_hist_keys2, dim3(g), dim3(256), 0, st, keys, n, s0, s1, hist);
}

void launch_hist_chunks(hipStream_t st, const uint64_t* keys, uint64_t n, uint32_t s0, uint32_t s1, uint32_t* cnt,
                        const uint32_t* redo, const uint32_t* top) {
    if (n == 0) return;
    unsigned g = blocks_for(n, 256 * 64);
    if (g > 512) g = 512;
    hipLaunchKernelGGL(k_hist_chunks, dim3(g), dim3(256), 0, st, keys, n, s0, s1, (n + SORT_TILE - 1) / SORT_TILE, cnt,
                       redo, top);
}

void launch_chunk_offsets(hipStream_t st, const uint32_t* cnt, uint64_t n, uint32_t* off1, uint32_t* off2,
                          ChunkTables tb1, ChunkTables tb2) {
    hipLaunchKernelGGL(k_chunk_offsets, dim3(1), dim3(256), 0, st, cnt, n, (n + SORT_TILE - 1) / SORT_TILE, off1, off2,
                       tb1.first_tile, tb1.ntiles, tb1.pos_begin, tb1.pos_end, tb2.first_tile, tb2.ntiles,
                       tb2.pos_begin, tb2.pos_end);
}

void launch_seg_hist_keys(hipStream_t st, const uint64_t* keys, uint64_t max_tiles, const uint32_t* ntiles,
                          const SegTiles& sg, uint32_t* hist) {
    if (!max_tiles) return;
    const unsigned g = max_tiles > 2048 ? 2048u : (unsigned)max_tiles;
    hipLaunchKernelGGL(k_seg_hist_keys, dim3(g), dim3(256), 0, st, keys, sg, ntiles, hist);
}

}  // namespace psi
