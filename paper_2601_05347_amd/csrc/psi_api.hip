// C ABI of the library: index lifetime, build, queries, inspection, timing.
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>

#include "psi_index.h"
#include "psi_update.h"

using namespace psi;

namespace psi {

psi_status hip_ok(hipError_t e) {
    if (e == hipSuccess) return PSI_OK;
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? PSI_E_NOMEM : PSI_E_HIP;
}

static psi_status last_launch() { return hip_ok(hipGetLastError()); }

bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return cs == hipStreamCaptureStatusActive;
}

psi_status ensure_q(psi_index ix, Buf& b, size_t need) {
    if (need <= b.bytes) return PSI_OK;
    if (capturing(ix->st)) return PSI_E_STATE;
    ++ix->gen;
    return b.ensure_q(need, ix->grave);
}

psi_status grow_keep_q(psi_index ix, Buf& b, size_t need) {
    if (need <= b.bytes) return PSI_OK;
    if (capturing(ix->st)) return PSI_E_STATE;
    ++ix->gen;
    return b.grow_keep_q(need, ix->st, ix->grave);
}

static void add(Bounds& a, const Bounds& d) {
    a.L += d.L;
    a.slot_top += d.slot_top;
    a.n_free += d.n_free;
    a.n_live += d.n_live;
    a.next_id += d.next_id;
}

static Bounds head_bounds(const DevTree& h) {
    Bounds b;
    b.L = h.L;
    b.slot_top = h.slot_top;
    b.n_free = h.n_free;
    b.n_live = h.n_live;
    b.next_id = h.next_id;
    return b;
}

void poll(psi_index ix) {
    if (capturing(ix->st)) return;
    while (!ix->inflight.empty()) {
        Inflight& f = ix->inflight.front();
        const hipError_t e = hipEventQuery(f.ev);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) (void)hipGetLastError();
        if (!f.stale) {
            ix->base = head_bounds(ix->mirror[f.slot]);
            ix->bucket_top = ix->mirror[f.slot].sort_top;
        }
        ix->ev_pool.push_back(f.ev);
        ix->inflight.pop_front();
    }
    // replaced blocks are freed in bunches (a free of device memory is a
    // synchronous call): when eight have gathered and the streams are idle
    if (ix->grave.size() >= 8 && ix->inflight.empty() && hipStreamQuery(ix->st) == hipSuccess &&
        (!ix->aux_st || hipStreamQuery(ix->aux_st) == hipSuccess)) {
        for (void* p : ix->grave) (void)hipFree(p);
        ix->grave.clear();
    }
}

psi_status settle(psi_index ix) {
    if (capturing(ix->st)) return PSI_E_STATE;
    psi_status s = hip_ok(hipStreamSynchronize(ix->st));
    if (s != PSI_OK) return s;
    if (ix->aux_st && (s = hip_ok(hipStreamSynchronize(ix->aux_st))) != PSI_OK) return s;
    for (Inflight& f : ix->inflight) ix->ev_pool.push_back(f.ev);
    ix->inflight.clear();
    for (void* p : ix->grave) (void)hipFree(p);
    ix->grave.clear();
    // the device's own answer (also after graph replays)
    if ((s = hip_ok(hipMemcpy(ix->mirror, ix->dev.p, DEVTREE_HEAD, hipMemcpyDeviceToHost))) != PSI_OK) return s;
    ix->base = head_bounds(ix->mirror[0]);
    ix->bucket_top = ix->mirror[0].sort_top;
    ix->unknown = false;
    return PSI_OK;
}

psi_status bounds(psi_index ix, Bounds* out) {
    if (ix->unknown) {
        psi_status s = settle(ix);
        if (s != PSI_OK) return s;
    }
    poll(ix);
    for (;;) {
        Bounds b = ix->base;
        for (const Inflight& f : ix->inflight)
            if (!f.stale) add(b, f.delta);
        // Worst cases add up when large updates are queued back to back, and
        // grids, scans and buffers follow the bound: with two or more updates
        // queued and the bound past 1.5 times the last known size, the oldest
        // is waited for (the device still has the others to run).
        const bool loose = b.L > ix->base.L + ix->base.L / 2 + (1u << 16) ||
                           b.slot_top > ix->base.slot_top + ix->base.slot_top / 2 + (1u << 16);
        if (!loose || ix->inflight.size() < 2 || capturing(ix->st)) {
            *out = b;
            return PSI_OK;
        }
        psi_status s = hip_ok(hipEventSynchronize(ix->inflight.front().ev));
        if (s != PSI_OK) return s;
        poll(ix);
    }
}

psi_status track_update(psi_index ix, const Bounds& delta) {
    if (capturing(ix->st)) return PSI_OK;  // replays are accounted for at launch
    if (ix->inflight.size() >= MIRROR_SLOTS) {
        // too many updates queued: wait for the oldest
        psi_status s = hip_ok(hipEventSynchronize(ix->inflight.front().ev));
        if (s != PSI_OK) return s;
        poll(ix);
    }
    Inflight f;
    f.delta = delta;
    f.slot = ix->mirror_next;
    ix->mirror_next = (ix->mirror_next + 1) % MIRROR_SLOTS;
    if (!ix->ev_pool.empty()) {
        f.ev = ix->ev_pool.back();
        ix->ev_pool.pop_back();
    } else {
        psi_status s = hip_ok(hipEventCreateWithFlags(&f.ev, hipEventDisableTiming));
        if (s != PSI_OK) return s;
    }
    psi_status s = hip_ok(hipMemcpyAsync(ix->mirror + f.slot, ix->dev.p, DEVTREE_HEAD, hipMemcpyDeviceToHost, ix->st));
    if (s == PSI_OK) s = hip_ok(hipEventRecord(f.ev, ix->st));
    if (s != PSI_OK) {
        ix->ev_pool.push_back(f.ev);
        return s;
    }
    ix->inflight.push_back(f);
    return PSI_OK;
}

psi_status readback(psi_index ix, const void* dev, size_t bytes) {
    if (capturing(ix->st)) return PSI_E_STATE;
    psi_status s = hip_ok(hipMemcpyAsync(ix->pinned, dev, bytes, hipMemcpyDeviceToHost, ix->st));
    if (s != PSI_OK) return s;
    return hip_ok(hipStreamSynchronize(ix->st));
}

// Stable LSD sort of (key, id) pairs; the result lands in sorter.k/i[*which].
// Passes: optionally the four id bytes first (so equal keys end up in id
// order whatever the input order), then the eight key bytes.
psi_status sort_pairs(psi_index ix, const uint64_t* kin, const uint32_t* iin, uint32_t id_base, uint64_t n,
                      bool id_digits, bool hist_ready, int* which, const char* fam, uint32_t key_shift0,
                      int key_passes, Sorter* sorter) {
    Sorter& S = sorter ? *sorter : ix->sorter;
    PassList pl{};
    pl.n = 0;
    if (id_digits)
        for (int b = 0; b < 4; ++b) { pl.src[pl.n] = 1; pl.shift[pl.n] = (uint8_t)(8 * b); ++pl.n; }
    for (int b = 0; b < key_passes; ++b) { pl.src[pl.n] = 0; pl.shift[pl.n] = (uint8_t)(key_shift0 + 8 * b); ++pl.n; }
    psi_status s;
    hipStream_t st = ix->st;
    const bool cap = capturing(st);
    if (n <= SORT_SMALL_MAX) {  // every pass in one workgroup's LDS, one launch
        if ((s = ensure_q(ix, S.k[0], std::max<uint64_t>(n, 1) * 8)) != PSI_OK) return s;
        if ((s = ensure_q(ix, S.i[0], std::max<uint64_t>(n, 1) * 4)) != PSI_OK) return s;
        ProfScope ps(ix, fam, n * 24 * pl.n);
        launch_sort_small(st, kin, iin, id_base, (uint32_t)n, pl, S.k[0].as<uint64_t>(), S.i[0].as<uint32_t>());
        *which = 0;
        return last_launch();
    }
    if ((s = ensure_q(ix, S.hist, MAX_PASSES * RADIX * 4)) != PSI_OK) return s;
    if ((s = ensure_q(ix, S.off, MAX_PASSES * RADIX * 4)) != PSI_OK) return s;
    if ((s = ensure_q(ix, S.ctr, MAX_PASSES * 4)) != PSI_OK) return s;
    for (int b = 0; b < 2; ++b) {
        if ((s = ensure_q(ix, S.k[b], n * 8)) != PSI_OK) return s;
        if ((s = ensure_q(ix, S.i[b], n * 4)) != PSI_OK) return s;
    }
    const uint64_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
    if (tiles * RADIX > S.status_words) {
        if ((s = ensure_q(ix, S.status, tiles * RADIX * 8)) != PSI_OK) return s;
        S.status_words = S.status.bytes / 8;
        launch_fill_u32(ix->st, S.status.as<uint32_t>(), S.status_words * 2, 0u);
    }
    if (!hist_ready) {
        launch_fill_u32(ix->st, S.hist.as<uint32_t>(), (uint64_t)pl.n * RADIX, 0u);
        ProfScope ps(ix, "hist", n * 12);
        launch_hist_pairs(ix->st, kin, iin, id_base, n, pl, S.hist.as<uint32_t>());
    } else if (id_digits) {
        return PSI_E_INTERNAL;
    }
    launch_digit_offsets(ix->st, pl.n, S.hist.as<uint32_t>(), S.off.as<uint32_t>());
    launch_fill_u32(ix->st, S.ctr.as<uint32_t>(), MAX_PASSES, 0u);
    const uint64_t* ksrc = kin;
    const uint32_t* isrc = iin;
    // one timing scope for all passes: an event pair per pass would space the
    // short passes of a small batch apart
    ProfScope ps(ix, fam, n * 24 * pl.n);
    for (int p = 0; p < pl.n; ++p) {
        const int dst = p & 1;
        if (++S.epoch >= (1u << 30)) {
            S.epoch = 1;
            launch_fill_u32(ix->st, S.status.as<uint32_t>(), S.status_words * 2, 0u);
        }
        // a graph replays the epoch it was captured with: clear the words first
        if (cap) launch_fill_u32(ix->st, S.status.as<uint32_t>(), tiles * RADIX * 2, 0u);
        launch_onesweep(ix->st, p == 0 && iin == nullptr, pl.src[p] == 1, ksrc, isrc, id_base,
                        S.k[dst].as<uint64_t>(), S.i[dst].as<uint32_t>(), n, pl.shift[p],
                        S.off.as<uint32_t>() + p * RADIX, S.status.as<uint64_t>(), S.ctr.as<uint32_t>() + p,
                        S.epoch, ix->err.as<uint32_t>());
        ksrc = S.k[dst].as<uint64_t>();
        isrc = S.i[dst].as<uint32_t>();
    }
    *which = (pl.n - 1) & 1;
    return last_launch();
}

// Build sort of n pairs (key, id_base + position): two global passes on the
// bucket bits [top, top + 16) (top = 16 below the largest key's leading bit,
// on the device), then every bucket (pairs equal in those bits) sorted by its
// low `top` bits in LDS; buckets too large for that take segmented global
// passes over the low bits. Same result as the eight-pass LSD sort: keys
// ascending, equal keys in id order. Nothing is read back: the digit counts
// were taken while encoding for the host's guess of top; if the true top
// differs they are taken again on the device, every later kernel reads top
// from the device, the passes whose tile counts depend on the data take tiles
// until none is left, and the big-bucket passes run over as many tiles as the
// device counted (none for most inputs).
constexpr uint64_t BUCKET_MIN_N = 1ull << 24;

// Counts, digit offsets and chunk tables of the two bucket passes, in one
// buffer: cnt [2][XCD_CHUNKS][256] first.
constexpr uint64_t XT_WORDS = 2 * XCD_CHUNKS * RADIX * 2 + XCD_CHUNKS * 4 + XCD_CHUNKS * 8 + 16;

psi_status bucket_sort(psi_index ix, const uint64_t* keys, uint32_t id_base, uint64_t n, uint32_t guess,
                       const uint64_t* kmax, int* which) {
    Sorter& S = ix->sorter;
    hipStream_t st = ix->st;
    psi_status s;
    if ((s = ensure_q(ix, S.off, MAX_PASSES * RADIX * 4)) != PSI_OK) return s;
    // tile counters: [0, 8) first pass, [8, 16) second pass, [16, 22) big buckets
    constexpr uint32_t CTR_WORDS = 2 * XCD_CHUNKS + 8;
    if ((s = ensure_q(ix, S.ctr, CTR_WORDS * 4)) != PSI_OK) return s;
    for (int b = 0; b < 2; ++b) {
        if ((s = ensure_q(ix, S.k[b], n * 8)) != PSI_OK) return s;
        if ((s = ensure_q(ix, S.i[b], n * 4)) != PSI_OK) return s;
    }
    const uint32_t nb = BUCKET_COUNT;
    const uint64_t T = (n + SORT_TILE - 1) / SORT_TILE;
    // big buckets hold more than BUCKET_MAX pairs each; their tiles number at
    // most T + (number of big buckets)
    const uint64_t nbig_max = std::min<uint64_t>(nb, n / (BUCKET_MAX + 1) + 1);
    const uint64_t btiles_max = T + nbig_max;
    auto ensure_status = [&](uint64_t tiles) -> psi_status {
        if (tiles * RADIX <= S.status_words) return PSI_OK;
        psi_status r = ensure_q(ix, S.status, tiles * RADIX * 8);
        if (r != PSI_OK) return r;
        S.status_words = S.status.bytes / 8;
        launch_fill_u32(st, S.status.as<uint32_t>(), S.status_words * 2, 0u);
        return PSI_OK;
    };
    auto next_epoch = [&]() {
        if (++S.epoch >= (1u << 30)) {
            S.epoch = 1;
            launch_fill_u32(st, S.status.as<uint32_t>(), S.status_words * 2, 0u);
        }
        return S.epoch;
    };
    const uint64_t tmpw = scan_tmp_words(nb);
    if ((s = ensure_q(ix, S.bk, ((uint64_t)nb * 5 + 1 + 2 + 2 + 2 * tmpw) * 4)) != PSI_OK) return s;
    uint32_t* bstart = S.bk.as<uint32_t>();  // nb + 1
    uint32_t* big = bstart + nb + 1;
    uint32_t* ntiles = big + nb;
    uint32_t* tile_off = ntiles + nb;
    uint32_t* big_idx = tile_off + nb;
    uint32_t* totals = big_idx + nb;  // 2: tiles of the big buckets, big buckets
    uint32_t* redo = totals + 2;      // 1
    uint32_t* tmp = redo + 2;  // 2 tmpw: the two scans of the big-bucket tables
    uint32_t* top = &ix->dt()->sort_top;
    if ((s = ensure_status(btiles_max + XCD_CHUNKS)) != PSI_OK) return s;
    if ((s = ensure_q(ix, S.xt, XT_WORDS * 4)) != PSI_OK) return s;
    const uint64_t seg_words = btiles_max * 2 + nbig_max * 2;
    if ((s = ensure_q(ix, S.bseg, seg_words * 4 + nbig_max * 8 + 8)) != PSI_OK) return s;
    if ((s = ensure_q(ix, S.shist, nbig_max * 8 * RADIX * 4)) != PSI_OK) return s;
    if ((s = ensure_q(ix, S.soff, nbig_max * 8 * RADIX * 4)) != PSI_OK) return s;
    uint32_t* cnt = S.xt.as<uint32_t>();             // [2][8][256]
    uint32_t* off1 = cnt + 2 * XCD_CHUNKS * RADIX;   // [8][256]
    uint32_t* off2 = off1 + XCD_CHUNKS * RADIX;      // [8][256]
    uint32_t* tw = off2 + XCD_CHUNKS * RADIX;        // first/ntiles of both passes
    uint64_t* tq = reinterpret_cast<uint64_t*>(S.xt.as<char>() + ((reinterpret_cast<char*>(tw + 4 * XCD_CHUNKS) - S.xt.as<char>() + 7) & ~(uint64_t)7));
    ChunkTables tb1{tw, tw + XCD_CHUNKS, tq, tq + XCD_CHUNKS};
    ChunkTables tb2{tw + 2 * XCD_CHUNKS, tw + 3 * XCD_CHUNKS, tq + 2 * XCD_CHUNKS, tq + 3 * XCD_CHUNKS};
    launch_fill_u32(st, S.ctr.as<uint32_t>(), CTR_WORDS, 0u);
    {
        // the counts were taken for `guess`; if the largest key says
        // otherwise, they are taken again for the true bucket bits
        ProfScope ps(ix, "hist", 0);
        launch_fix_top(st, kmax, guess, top, redo);
        st_fill_gated(st, cnt, 2 * XCD_CHUNKS * RADIX, 0u, redo);
        launch_hist_chunks(st, keys, n, 0, 0, cnt, redo, top);
        launch_chunk_offsets(st, cnt, n, off1, off2, tb1, tb2);
    }
    if ((s = last_launch()) != PSI_OK) return s;
    const XcdChunks xc1{tb1.first_tile, tb1.ntiles, tb1.pos_begin, tb1.pos_end};
    const XcdChunks xc2{tb2.first_tile, tb2.ntiles, tb2.pos_begin, tb2.pos_end};
    const uint32_t per_chunk = (uint32_t)((T + XCD_CHUNKS - 1) / XCD_CHUNKS);
    {
        // 8 B key read (ids implicit), 12 B written
        ProfScope ps(ix, "radix_first", n * 20);
        launch_onesweep_xcd(st, true, keys, nullptr, id_base, S.k[0].as<uint64_t>(), S.i[0].as<uint32_t>(), n, 0,
                            off1, S.status.as<uint64_t>(), S.ctr.as<uint32_t>(), next_epoch(), ix->err.as<uint32_t>(),
                            xc1, per_chunk, top, false);
    }
    {
        // the second pass's chunks have data-dependent sizes: a workgroup
        // per tile of a balanced chunk, then an overflow launch for the rest
        ProfScope ps(ix, "radix_pass", n * 24);
        launch_onesweep_xcd(st, false, S.k[0].as<uint64_t>(), S.i[0].as<uint32_t>(), 0, S.k[1].as<uint64_t>(),
                            S.i[1].as<uint32_t>(), n, 8, off2, S.status.as<uint64_t>(),
                            S.ctr.as<uint32_t>() + XCD_CHUNKS, next_epoch(), ix->err.as<uint32_t>(), xc2, per_chunk,
                            top, true);
    }
    uint64_t* K = S.k[1].as<uint64_t>();
    uint32_t* I = S.i[1].as<uint32_t>();
    // timing scopes: the light variant alone (it sorts all but the rare
    // buckets of more than BUCKET_SMALL pairs, whose bytes it is charged)
    {
        ProfScope ps(ix, "bucket_starts", (uint64_t)nb * 8);
        launch_bucket_starts(st, K, n, top, bstart, nb);
    }
    {
        ProfScope ps(ix, "local_sort", n * 24);
        launch_local_sort(st, K, I, bstart, nb, top, big, ix->err.as<uint32_t>(), false);
    }
    {
        ProfScope ps(ix, "local_sort_wide", 0);
        launch_local_sort(st, K, I, bstart, nb, top, big, ix->err.as<uint32_t>(), true);
    }
    if (n > (uint64_t)BUCKET_MAX) {
        // one workgroup per CU (none of its buckets in range for uniform data
        // below about 2.5e8 points)
        ProfScope ps(ix, "local_sort_huge", 0);
        launch_local_sort_huge(st, K, I, bstart, nb, big);
    }
    launch_big_tables(st, bstart, big, nb, ntiles, tile_off, big_idx, totals, tmp);
    *which = 1;
    // big buckets: segmented passes over their tiles only (k/i[1] -> [0] ->
    // ... -> [1]), six of them (top <= 47: the low bits take at most six
    // 8-bit digits; a pass over bits at or above top is constant inside a
    // bucket and changes nothing). With no big bucket every launch below
    // finds no tile and exits.
    uint64_t* seg_begin = S.bseg.as<uint64_t>();
    uint32_t* tile_seg = reinterpret_cast<uint32_t*>(seg_begin + nbig_max);
    uint32_t* tile_beg = tile_seg + btiles_max;
    uint32_t* seg_first = tile_beg + btiles_max;
    uint32_t* seg_end = seg_first + nbig_max;
    SegTiles sg{tile_seg, tile_beg, seg_first, seg_end, 8 * RADIX};
    constexpr int NP = 6;
    const uint64_t grid = std::min<uint64_t>(btiles_max, 1024);
    ProfScope ps(ix, "radix_big", 0);
    launch_big_fill(st, bstart, big, big_idx, tile_off, nb, sg, seg_begin);
    launch_zero_counted(st, S.shist.as<uint32_t>(), 8 * RADIX, totals + 1, nbig_max);
    launch_seg_hist_keys(st, K, btiles_max, totals, sg, S.shist.as<uint32_t>());
    launch_seg_digit_offsets(st, (uint32_t)nbig_max, S.shist.as<uint32_t>(), seg_begin, S.soff.as<uint32_t>(),
                             totals + 1);
    for (int p = 0; p < NP; ++p) {
        const int src = (p & 1) ? 0 : 1, dst = 1 - src;
        launch_onesweep(st, false, false, S.k[src].as<uint64_t>(), S.i[src].as<uint32_t>(), 0, S.k[dst].as<uint64_t>(),
                        S.i[dst].as<uint32_t>(), n, 8 * p, S.soff.as<uint32_t>() + p * RADIX, S.status.as<uint64_t>(),
                        S.ctr.as<uint32_t>() + 2 * XCD_CHUNKS + p, next_epoch(), ix->err.as<uint32_t>(), &sg, grid,
                        totals);
    }
    return last_launch();
}

// Node levels over the current directory (the layout the device state
// holds), from the level just above the leaves up to the root. The node
// buffers and the packed boxes are sized for up to L_bound leaves and the
// launches cover the height of L_bound leaves; levels above the tree's real
// height do nothing.
psi_status build_nodes(psi_index ix, uint64_t L_bound) {
    uint64_t inner_n = 0;
    uint32_t h = 0;
    for (uint64_t n = L_bound; n > 1; ++h) {
        n = (n + ix->B - 1) / ix->B;
        inner_n += n;
    }
    if (h + 1 > (uint32_t)MAX_LEVELS) return PSI_E_INTERNAL;
    psi_status s;
    if ((s = grow_keep_q(ix, ix->inner, std::max<uint64_t>(inner_n, 1) * sizeof(NodeRec))) != PSI_OK) return s;
    // the packed boxes follow on the next kNN (sized here: a captured kNN
    // cannot allocate)
    ix->boxes_fresh = false;
    if ((s = ensure_q(ix, ix->cinner, std::max<uint64_t>(inner_n, 1) * 16)) != PSI_OK) return s;
    if ((s = ensure_q(ix, ix->cleaf, std::max<uint64_t>(L_bound, 1) * 16)) != PSI_OK) return s;
    ix->L_cap = std::max(ix->L_cap, L_bound);
    ProfScope ps(ix, "nodes", inner_n * 32 + L_bound * 32);
    launch_node_levels(ix->st, ix->D, ix->dt(), dirs_of(ix), L_bound, ix->inner.as<NodeRec>(), ix->B);
    const uint64_t ns = (L_bound + PSAMPLE - 1) / PSAMPLE + 1;
    if ((s = ensure_q(ix, ix->psample, ns * 16)) != PSI_OK) return s;
    launch_pivot_sample(ix->st, ix->dt(), dirs_of(ix), ix->psample.as<uint4>(), ns);
    return last_launch();
}

// Curve keys of n points (into `keys`) and the pairs (key, id_base +
// position) sorted by key, then id, into sorter.k/i[*which] (Alg. 3's sort
// step). Requires n > 0.
psi_status encode_sort(psi_index ix, const uint32_t* d_pts, uint64_t n, uint64_t* keys, uint32_t id_base,
                       int* which) {
    psi_status s;
    Sorter& S = ix->sorter;
    if ((s = ensure_q(ix, S.hist, MAX_PASSES * RADIX * 4)) != PSI_OK) return s;
    launch_fill_u32(ix->st, S.hist.as<uint32_t>(), 8 * RADIX, 0u);
    const bool two_level = ((ix->flags & PSI_FLAG_SORT_BUCKETS) ||
                            (n >= BUCKET_MIN_N && !(ix->flags & PSI_FLAG_SORT_LSD))) &&
                           !capturing(ix->st);
    int w = 0;
    if (two_level) {
        // keys and their maximum; the bucket bits are the 16 below its leading
        // bit. The bucket digits are counted while encoding for a guess of
        // those bits (the last build's, once the host has seen it, else the
        // top of the key width); a wrong guess costs one more read of the
        // keys on the device, never a different result.
        if ((s = ensure_q(ix, S.kmax, 8)) != PSI_OK) return s;
        if ((s = ensure_q(ix, S.xt, XT_WORDS * 4)) != PSI_OK) return s;
        const uint32_t guess = ix->bucket_top <= 48 ? ix->bucket_top : (ix->D == 2 ? 62u : 63u) - 16u;
        launch_fill_u32(ix->st, S.kmax.as<uint32_t>(), 2, 0u);
        launch_fill_u32(ix->st, S.xt.as<uint32_t>(), 2 * XCD_CHUNKS * RADIX, 0u);
        {
            ProfScope ps(ix, "encode_hist", n * (4 * ix->D + 8));
            launch_encode_chunks(ix->st, ix->D, ix->curve, d_pts, n, keys, ix->err.as<uint32_t>(),
                                 S.kmax.as<uint64_t>(), guess, S.xt.as<uint32_t>());
        }
        s = bucket_sort(ix, keys, id_base, n, guess, S.kmax.as<uint64_t>(), &w);
    } else {
        {
            ProfScope ps(ix, "encode_hist", n * (4 * ix->D + 8));
            launch_encode_hist(ix->st, ix->D, ix->curve, d_pts, n, keys, S.hist.as<uint32_t>(),
                               ix->err.as<uint32_t>());
        }
        s = sort_pairs(ix, keys, nullptr, id_base, n, false, true, &w, "radix_pass");
    }
    *which = w;
    return s;
}

Dirs dirs_of(psi_index ix) {
    Dirs d;
    for (int b = 0; b < 2; ++b) {
        d.leaf[b] = ix->leaf[b].as<NodeRec>();
        d.pkey[b] = ix->pkey[b].as<uint64_t>();
        d.pid[b] = ix->pid[b].as<uint32_t>();
    }
    return d;
}

// Directory buffers for up to `leaves` leaves each, contents kept; the device
// state learns the new addresses in stream order.
psi_status ensure_dirs(psi_index ix, uint64_t leaves) {
    const uint64_t Lc = std::max<uint64_t>(leaves, 1);
    const void* before[6] = {ix->leaf[0].p, ix->leaf[1].p, ix->pkey[0].p, ix->pkey[1].p, ix->pid[0].p, ix->pid[1].p};
    psi_status s;
    for (int b = 0; b < 2; ++b) {
        if ((s = grow_keep_q(ix, ix->leaf[b], Lc * sizeof(NodeRec))) != PSI_OK) return s;
        if ((s = grow_keep_q(ix, ix->pkey[b], Lc * 8)) != PSI_OK) return s;
        if ((s = grow_keep_q(ix, ix->pid[b], Lc * 4)) != PSI_OK) return s;
    }
    const void* after[6] = {ix->leaf[0].p, ix->leaf[1].p, ix->pkey[0].p, ix->pkey[1].p, ix->pid[0].p, ix->pid[1].p};
    if (std::memcmp(before, after, sizeof before) != 0)
        st_set_dirs(ix->st, ix->dt(), ix->leaf[0].as<NodeRec>(), ix->leaf[1].as<NodeRec>(), ix->pkey[0].as<uint64_t>(),
                    ix->pkey[1].as<uint64_t>(), ix->pid[0].as<uint32_t>(), ix->pid[1].as<uint32_t>());
    return last_launch();
}

// Fresh build of the n points (Alg. 3): ids 0 .. n - 1, replacing the
// contents. The leaf count is known on the host, and so is every size of
// the new state.
psi_status do_build(psi_index ix, const uint32_t* d_pts, uint64_t n) {
    psi_status s;
    ++ix->gen;
    // updates still in flight describe the state this build replaces
    for (Inflight& f : ix->inflight) f.stale = true;
    const uint64_t L = (n + ix->phi - 1) / ix->phi;
    if ((s = ensure_q(ix, ix->idkey, std::max<uint64_t>(n, 1) * 8)) != PSI_OK) return s;
    if ((s = ensure_dirs(ix, L)) != PSI_OK) return s;
    if ((s = ensure_q(ix, ix->slots, std::max<uint64_t>(L, 1) * ix->slot_words() * 4)) != PSI_OK) return s;
    if (n > 0) {
        int w = 0;
        if ((s = encode_sort(ix, d_pts, n, ix->idkey.as<uint64_t>(), 0, &w)) != PSI_OK) return s;
        Sorter& S = ix->sorter;
        ProfScope ps(ix, "leaf_fill", n * (12 + 4 * (uint64_t)(ix->D + 1)) + L * 44);
        launch_build_leaves(ix->st, ix->D, ix->curve, S.k[w].as<uint64_t>(), S.i[w].as<uint32_t>(), n, L, ix->C,
                            ix->slots.as<uint32_t>(), ix->pkey[0].as<uint64_t>(), ix->pid[0].as<uint32_t>(),
                            ix->leaf[0].as<NodeRec>());
    }
    st_commit_build(ix->st, ix->dt(), n, L, 0, (uint32_t)n, ix->B);
    if ((s = last_launch()) != PSI_OK) return s;
    Bounds b;
    b.L = L;
    b.slot_top = L;
    b.n_free = 0;
    b.n_live = n;
    b.next_id = n;
    ix->base = b;
    if ((s = build_nodes(ix, L)) != PSI_OK) return s;
    // mirror the head too: the next build learns the bucket bits from it
    return track_update(ix, Bounds{});
}

// Processing order of a query batch: the batch's positions sorted by the
// curve key of each query point (or box centre), so that the queries one
// wave handles lie close together in space and share tree nodes and leaves.
// Query points are also range-checked here (errors are latched).
static const uint64_t ORDER_MIN = 4096;

psi_status query_order(psi_index ix, const uint32_t* d_items, uint64_t n, bool boxes, const uint32_t** order) {
    *order = nullptr;
    const bool sort = n >= ORDER_MIN && !(ix->flags & PSI_FLAG_INPUT_ORDER);
    if (boxes && !sort) return PSI_OK;
    psi_status s;
    if ((s = ensure_q(ix, ix->qkeys, n * 8)) != PSI_OK) return s;
    uint64_t* keys = ix->qkeys.as<uint64_t>();
    {
        ProfScope ps(ix, "order", n * (boxes ? 8ull * ix->D : 4ull * ix->D) + n * 8);
        if (boxes) launch_encode_boxes(ix->st, ix->D, ix->curve, d_items, n, keys);
        else launch_encode(ix->st, ix->D, ix->curve, d_items, n, keys, ix->err.as<uint32_t>());
    }
    if (!sort) return last_launch();
    // Only locality matters here (results never depend on the order): the top
    // 24 bits of the curve key (cells of about 2^-24 of the domain) in three
    // passes instead of all 64 bits in eight.
    int w = 0;
    const uint32_t kb = ix->D == 2 ? 62u : 63u;
    const uint32_t ob = ix->order_bits;
    if ((s = sort_pairs(ix, keys, nullptr, 0, n, false, false, &w, "radix_order", kb - ob, (int)(ob / 8),
                        &ix->qsorter)) !=
        PSI_OK)
        return s;
    *order = ix->qsorter.i[w].as<uint32_t>();
    return last_launch();
}

}  // namespace psi

namespace psi {

TreeView exact_view(psi_index ix, std::vector<LevelInfo>* lv) {
    DevTree h{};
    (void)hipMemcpy(&h, ix->dev.p, sizeof(DevTree), hipMemcpyDeviceToHost);
    TreeView t{};
    t.inner = ix->inner.as<NodeRec>();
    t.leaf = h.leaf[h.cur];
    t.cinner = ix->cinner.as<uint4>();
    t.cleaf = ix->cleaf.as<uint4>();
    t.pkey = h.pkey[h.cur];
    t.slots = ix->slots.as<uint32_t>();
    t.h = h.h;
    t.B = ix->B;
    t.C = ix->C;
    t.L = h.L;
    t.dt = nullptr;
    if (lv) lv->assign(h.lv, h.lv + (h.L ? h.h + 1 : 0));
    return t;
}

}  // namespace psi

psi::TreeView psi_index_s::view() const {
    psi::TreeView t{};
    t.inner = inner.as<psi::NodeRec>();
    t.leaf = leaf[0].as<psi::NodeRec>();  // the kernels pick the current buffer by dt->cur
    t.leaf_alt = leaf[1].as<psi::NodeRec>();
    t.cinner = cinner.as<uint4>();
    t.cleaf = cleaf.as<uint4>();
    t.pkey = pkey[0].as<uint64_t>();
    t.pkey_alt = pkey[1].as<uint64_t>();
    t.slots = slots.as<uint32_t>();
    t.h = 0;
    t.B = B;
    t.C = C;
    t.L = 0;
    t.dt = dt();
    return t;
}

namespace {

// Graphs: which indexes a capture touched, at which generation. A replay is
// refused when an index changed on the host since (an eager update, a buffer
// that grew: the graph would read a stale directory or freed memory), and a
// replay that runs updates leaves the host's view of the sizes unknown until
// the next wait.
struct CapRec {
    psi_index ix;
    uint64_t gen;
    bool upd;
};
std::mutex g_mu;
std::map<hipStream_t, std::vector<CapRec>> g_cap;
std::set<psi_index> g_live;

void note_capture(psi_index ix, bool upd) {
    if (!capturing(ix->st)) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cap.find(ix->st);
    if (it == g_cap.end()) return;
    for (CapRec& r : it->second)
        if (r.ix == ix) {
            r.upd = r.upd || upd;
            return;
        }
    it->second.push_back({ix, 0, upd});
}

}  // namespace

extern "C" {

const char* psi_status_str(psi_status s) {
    switch (s) {
        case PSI_OK: return "ok";
        case PSI_E_ARG: return "invalid argument";
        case PSI_E_RANGE: return "coordinate out of range";
        case PSI_E_NOMEM: return "out of device memory";
        case PSI_E_CAPACITY: return "id space exhausted or reserved capacity exceeded";
        case PSI_E_HIP: return "HIP runtime error";
        case PSI_E_STATE: return "invalid state";
        case PSI_E_INTERNAL: return "internal consistency check failed";
    }
    return "unknown status";
}

psi_status psi_create(const psi_params* prm, void* hip_stream, psi_index* out) {
    if (!prm || !out) return PSI_E_ARG;
    *out = nullptr;
    if ((prm->dim != 2 && prm->dim != 3) || prm->curve > 1 || prm->leaf_size < 2 || prm->leaf_size > 32 ||
        prm->fanout < 2 || prm->fanout > 32 || (prm->flags & ~(uint32_t)(PSI_FLAG_INPUT_ORDER | PSI_FLAG_KNN_NEAREST_FIRST | PSI_FLAG_SORT_BUCKETS |
                                  PSI_FLAG_SORT_LSD | PSI_FLAG_SORTED_LEAVES)) != 0 ||
        (prm->flags & (PSI_FLAG_SORT_BUCKETS | PSI_FLAG_SORT_LSD)) == (PSI_FLAG_SORT_BUCKETS | PSI_FLAG_SORT_LSD))
        return PSI_E_ARG;
    psi_index ix = new (std::nothrow) psi_index_s;
    if (!ix) return PSI_E_NOMEM;
    ix->D = (int)prm->dim;
    ix->curve = (int)prm->curve;
    ix->phi = prm->leaf_size;
    ix->C = (2 * prm->leaf_size + 3) & ~3u;
    ix->B = prm->fanout;
    ix->flags = prm->flags;
    ix->st = static_cast<hipStream_t>(hip_stream);
    psi_status s = ix->err.ensure(64);
    if (s == PSI_OK) s = ix->dev.ensure(sizeof(DevTree));
    if (s == PSI_OK) s = hip_ok(hipHostMalloc(&ix->pinned, 4096, hipHostMallocDefault));
    if (s == PSI_OK)
        s = hip_ok(hipHostMalloc(reinterpret_cast<void**>(&ix->mirror), MIRROR_SLOTS * sizeof(DevTree),
                                 hipHostMallocDefault));
    if (s == PSI_OK) {
        launch_fill_u32(ix->st, ix->err.as<uint32_t>(), 16, 0u);
        st_set_dirs(ix->st, ix->dt(), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
        st_reset(ix->st, ix->dt(), ix->B);
        s = hip_ok(hipGetLastError());
    }
    if (s == PSI_OK) s = hip_ok(hipStreamSynchronize(ix->st));
    if (s != PSI_OK) {
        if (ix->pinned) (void)hipHostFree(ix->pinned);
        if (ix->mirror) (void)hipHostFree(ix->mirror);
        delete ix;
        return s;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(ix);
    }
    *out = ix;
    return PSI_OK;
}

psi_status psi_destroy(psi_index ix) {
    if (!ix) return PSI_E_ARG;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.erase(ix);
    }
    (void)hipStreamSynchronize(ix->st);
    for (void* p : ix->grave) (void)hipFree(p);
    for (Inflight& f : ix->inflight) (void)hipEventDestroy(f.ev);
    for (hipEvent_t e : ix->ev_pool) (void)hipEventDestroy(e);
    if (ix->pinned) (void)hipHostFree(ix->pinned);
    if (ix->mirror) (void)hipHostFree(ix->mirror);
    delete ix;
    return PSI_OK;
}

psi_status psi_set_stream(psi_index ix, void* hip_stream) {
    if (!ix) return PSI_E_ARG;
    psi_status s = settle(ix);
    ix->st = static_cast<hipStream_t>(hip_stream);
    return s;
}

psi_status psi_build(psi_index ix, const uint32_t* d_pts, uint64_t n) {
    if (!ix || (n && !d_pts)) return PSI_E_ARG;
    if (n > 0xFFFFFFFFull) return PSI_E_CAPACITY;
    note_capture(ix, true);
    psi_status s = do_build(ix, d_pts, n);
    if (s == PSI_OK && !capturing(ix->st)) ix->unknown = false;
    return s;
}

psi_status psi_batch_insert(psi_index ix, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids) {
    if (!ix || (m && !d_pts)) return PSI_E_ARG;
    if (m == 0) return PSI_OK;
    Bounds u;
    psi_status s = bounds(ix, &u);
    if (s != PSI_OK) return s;
    if (u.next_id + m > 0xFFFFFFFFull) return PSI_E_CAPACITY;
    note_capture(ix, true);
    return do_insert(ix, d_pts, m, d_new_ids);
}

psi_status psi_batch_delete(psi_index ix, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted) {
    if (!ix || (m && !d_ids)) return PSI_E_ARG;
    if (m > 0xFFFFFFFFull) return PSI_E_ARG;
    note_capture(ix, true);
    return do_delete(ix, d_ids, m, d_ndeleted);
}

psi_status psi_knn(psi_index ix, const uint32_t* d_q, uint64_t nq, uint32_t k, uint32_t* d_ids, uint64_t* d_d2) {
    if (!ix || k == 0 || k > 128 || (nq && (!d_q || !d_ids || !d_d2))) return PSI_E_ARG;
    if (nq == 0) return PSI_OK;
    note_capture(ix, false);
    const uint32_t* order = nullptr;
    psi_status s = query_order(ix, d_q, nq, false, &order);
    if (s != PSI_OK) return s;
    // The box tests read the packed boxes: rewritten after the tree changed,
    // and always inside a captured graph (a replay may follow updates). The
    // counts come from the device state, the grids from the buffers' size.
    const bool cap = capturing(ix->st);
    if (!ix->boxes_fresh || cap) {
        const uint64_t nl = ix->cleaf.bytes / 16, ni = ix->cinner.bytes / 16;
        ProfScope pb(ix, "pack_boxes", (ix->L_cap * 2) * 48);
        launch_pack_tree(ix->st, ix->D, ix->dt(), dirs_of(ix), true, nullptr, ix->cleaf.as<uint4>(), nl);
        launch_pack_tree(ix->st, ix->D, ix->dt(), dirs_of(ix), false, ix->inner.as<NodeRec>(), ix->cinner.as<uint4>(), ni);
        if (!cap) ix->boxes_fresh = true;
    }
    // the tree is never taller than one over the leaves the node buffers hold
    uint32_t hcap = 0;
    for (uint64_t n = ix->L_cap; n > 1; ++hcap) n = (n + ix->B - 1) / ix->B;
    ProfScope ps(ix, "knn", nq * (4ull * ix->D + 12ull * k));
    launch_knn(ix->st, ix->D, ix->view(), d_q, ix->qkeys.as<uint64_t>(), nq, order, k,
               (ix->flags & PSI_FLAG_KNN_NEAREST_FIRST) ? 1 : 0, hcap, ix->knn_tune, ix->err.as<uint32_t>(),
               ix->qstats_on ? ix->qstats.as<unsigned long long>() : nullptr, d_ids, d_d2);
    return last_launch();
}

psi_status psi_range_count(psi_index ix, const uint32_t* d_boxes, uint64_t nb, uint64_t* d_counts) {
    if (!ix || (nb && (!d_boxes || !d_counts))) return PSI_E_ARG;
    if (nb == 0) return PSI_OK;
    note_capture(ix, false);
    const uint32_t* order = nullptr;
    psi_status s = query_order(ix, d_boxes, nb, true, &order);
    if (s != PSI_OK) return s;
    ProfScope ps(ix, "range_count", nb * (8ull * ix->D + 8));
    launch_range_count(ix->st, ix->D, ix->view(), d_boxes, nb, order, d_counts);
    return last_launch();
}

psi_status psi_range_report(psi_index ix, const uint32_t* d_boxes, uint64_t nb, const uint64_t* d_offsets,
                            uint32_t* d_ids) {
    if (!ix || (nb && (!d_boxes || !d_offsets))) return PSI_E_ARG;
    if (nb == 0) return PSI_OK;
    note_capture(ix, false);
    const uint32_t* order = nullptr;
    psi_status s = query_order(ix, d_boxes, nb, true, &order);
    if (s != PSI_OK) return s;
    ProfScope ps(ix, "range_report", nb * (8ull * ix->D + 16));
    launch_range_report(ix->st, ix->D, ix->view(), d_boxes, nb, order, d_offsets, d_ids);
    return last_launch();
}

psi_status psi_sync(psi_index ix) {
    if (!ix) return PSI_E_ARG;
    psi_status s = settle(ix);
    if (s != PSI_OK) return s;
    uint32_t e = 0;
    if ((s = hip_ok(hipMemcpy(&e, ix->err.p, 4, hipMemcpyDeviceToHost))) != PSI_OK) return s;
    if (e) {
        launch_fill_u32(ix->st, ix->err.as<uint32_t>(), 1, 0u);
        (void)hipStreamSynchronize(ix->st);
        if (e & ERR_RANGE) return PSI_E_RANGE;
        if (e & ERR_CAPACITY) return PSI_E_CAPACITY;
        return PSI_E_INTERNAL;
    }
    return PSI_OK;
}

psi_status psi_size(psi_index ix, uint64_t* h_n_live) {
    if (!ix || !h_n_live) return PSI_E_ARG;
    psi_status s = psi_sync(ix);
    *h_n_live = ix->base.n_live;
    return s;
}

psi_status psi_next_id(psi_index ix, uint32_t* h_next_id) {
    if (!ix || !h_next_id) return PSI_E_ARG;
    psi_status s = settle(ix);
    *h_next_id = (uint32_t)ix->base.next_id;
    return s;
}

psi_status psi_export(psi_index ix, uint64_t* d_keys, uint32_t* d_ids, uint32_t* d_pts) {
    if (!ix) return PSI_E_ARG;
    psi_status s = settle(ix);
    if (s != PSI_OK) return s;
    const TreeView t = exact_view(ix);
    if (t.L == 0) return PSI_OK;
    if ((s = ensure_q(ix, ix->scr.a, (t.L + 1) * 8)) != PSI_OK) return s;
    if ((s = ensure_q(ix, ix->scr.b, (2 * t.L + scan_tmp_words(t.L) + 4) * 8)) != PSI_OK) return s;
    launch_leaf_offsets(ix->st, t.leaf, t.L, ix->scr.a.as<uint64_t>(), ix->scr.b.as<uint64_t>());
    launch_export_sorted(ix->st, ix->D, ix->curve, t, ix->scr.a.as<uint64_t>(), d_keys, d_ids, d_pts);
    return last_launch();
}

psi_status psi_export_leaves(psi_index ix, uint32_t* d_ids, uint32_t* d_pts) {
    if (!ix) return PSI_E_ARG;
    psi_status s = settle(ix);
    if (s != PSI_OK) return s;
    const TreeView t = exact_view(ix);
    if (t.L == 0) return PSI_OK;
    if ((s = ensure_q(ix, ix->scr.a, (t.L + 1) * 8)) != PSI_OK) return s;
    if ((s = ensure_q(ix, ix->scr.b, (2 * t.L + scan_tmp_words(t.L) + 4) * 8)) != PSI_OK) return s;
    launch_leaf_offsets(ix->st, t.leaf, t.L, ix->scr.a.as<uint64_t>(), ix->scr.b.as<uint64_t>());
    launch_export_raw(ix->st, ix->D, t, ix->scr.a.as<uint64_t>(), d_ids, d_pts);
    return last_launch();
}

psi_status psi_shape(psi_index ix, uint64_t* h_n_leaves, uint32_t* h_height, uint64_t* h_level_sizes) {
    if (!ix || !h_n_leaves || !h_height) return PSI_E_ARG;
    psi_status s = settle(ix);
    if (s != PSI_OK) return s;
    std::vector<LevelInfo> lv;
    const TreeView t = exact_view(ix, &lv);
    *h_n_leaves = t.L;
    *h_height = t.h;
    if (h_level_sizes)
        for (uint32_t l = 0; l < lv.size(); ++l) h_level_sizes[l] = lv[l].n;
    return PSI_OK;
}

psi_status psi_export_structure(psi_index ix, uint64_t* d_piv_key, uint32_t* d_piv_id, uint32_t* d_leaf_cnt,
                                uint32_t* d_leaf_lo, uint32_t* d_leaf_hi, uint32_t* d_node_lo, uint32_t* d_node_hi,
                                uint64_t* d_node_cnt) {
    if (!ix) return PSI_E_ARG;
    psi_status s = settle(ix);
    if (s != PSI_OK) return s;
    DevTree h{};
    if ((s = hip_ok(hipMemcpy(&h, ix->dev.p, sizeof(DevTree), hipMemcpyDeviceToHost))) != PSI_OK) return s;
    const TreeView t = exact_view(ix);
    launch_export_structure(ix->st, ix->D, t, h.L ? h.n_inner : 0, h.pkey[h.cur], h.pid[h.cur], d_piv_key, d_piv_id,
                            d_leaf_cnt, d_leaf_lo, d_leaf_hi, d_node_lo, d_node_hi, d_node_cnt);
    return last_launch();
}

psi_status psi_encode(uint32_t dim, uint32_t curve, const uint32_t* d_pts, uint64_t n, uint64_t* d_keys,
                      void* hip_stream) {
    if ((dim != 2 && dim != 3) || curve > 1 || (n && (!d_pts || !d_keys))) return PSI_E_ARG;
    if (n == 0) return PSI_OK;
    Buf err;
    psi_status s = err.ensure(4);
    if (s != PSI_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    launch_fill_u32(st, err.as<uint32_t>(), 1, 0u);
    launch_encode(st, (int)dim, (int)curve, d_pts, n, d_keys, err.as<uint32_t>());
    uint32_t e = 0;
    if ((s = hip_ok(hipMemcpyAsync(&e, err.p, 4, hipMemcpyDeviceToHost, st))) != PSI_OK) return s;
    if ((s = hip_ok(hipStreamSynchronize(st))) != PSI_OK) return s;
    return e ? PSI_E_RANGE : PSI_OK;
}

psi_status psi_sort_pairs(const uint64_t* d_keys, const uint32_t* d_ids, uint64_t n, uint64_t* d_keys_out,
                          uint32_t* d_ids_out, void* hip_stream) {
    if (n && (!d_keys || !d_ids || !d_keys_out || !d_ids_out)) return PSI_E_ARG;
    if (n > 0xFFFFFFFFull) return PSI_E_ARG;
    if (n == 0) return PSI_OK;
    psi_params prm{2, 0, 32, 8, 0};
    psi_index ix = nullptr;
    psi_status s = psi_create(&prm, hip_stream, &ix);
    if (s != PSI_OK) return s;
    int w = 0;
    s = sort_pairs(ix, d_keys, d_ids, 0, n, true, false, &w, "radix_pass");
    if (s == PSI_OK) s = hip_ok(hipMemcpyAsync(d_keys_out, ix->sorter.k[w].p, n * 8, hipMemcpyDeviceToDevice, ix->st));
    if (s == PSI_OK) s = hip_ok(hipMemcpyAsync(d_ids_out, ix->sorter.i[w].p, n * 4, hipMemcpyDeviceToDevice, ix->st));
    psi_status e = psi_sync(ix);
    if (s == PSI_OK) s = e;
    psi_destroy(ix);
    return s;
}

struct psi_graph_s {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    std::vector<CapRec> idx;  // indexes the captured calls touched
};

psi_status psi_graph_begin(void* hip_stream) {
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cap[st].clear();
    }
    return hip_ok(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
}

psi_status psi_graph_end(void* hip_stream, psi_graph* out) {
    if (!out) return PSI_E_ARG;
    *out = nullptr;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    std::vector<CapRec> recs;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cap.find(st);
        if (it != g_cap.end()) {
            recs = it->second;
            g_cap.erase(it);
        }
    }
    for (CapRec& r : recs) {
        r.gen = r.ix->gen;
        // the captured updates did not run: the host's view of the sizes is
        // only a bound of what a replay will leave
        if (r.upd) r.ix->unknown = true;
    }
    psi_graph g = new (std::nothrow) psi_graph_s;
    hipGraph_t graph = nullptr;
    psi_status s = hip_ok(hipStreamEndCapture(st, &graph));
    if (!g) {
        if (graph) (void)hipGraphDestroy(graph);
        return PSI_E_NOMEM;
    }
    if (s == PSI_OK) s = hip_ok(hipGraphInstantiate(&g->e, graph, nullptr, nullptr, 0));
    g->g = graph;
    g->idx = recs;
    if (s != PSI_OK) {
        if (g->g) (void)hipGraphDestroy(g->g);
        delete g;
        return s;
    }
    *out = g;
    return PSI_OK;
}

psi_status psi_graph_launch(psi_graph g, void* hip_stream) {
    if (!g) return PSI_E_ARG;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const CapRec& r : g->idx)
            if (!g_live.count(r.ix) || r.ix->gen != r.gen) return PSI_E_STATE;
    }
    psi_status s = hip_ok(hipGraphLaunch(g->e, static_cast<hipStream_t>(hip_stream)));
    for (const CapRec& r : g->idx)
        if (r.upd) {
            r.ix->unknown = true;
            r.ix->boxes_fresh = false;
        }
    return s;
}

psi_status psi_graph_destroy(psi_graph g) {
    if (!g) return PSI_E_ARG;
    if (g->e) (void)hipGraphExecDestroy(g->e);
    if (g->g) (void)hipGraphDestroy(g->g);
    delete g;
    return PSI_OK;
}

psi_status psi_set_tuning(psi_index ix, const psi_tuning* t) {
    if (!ix || !t) return PSI_E_ARG;
    if (t->knn_seed_leaves < 1 || t->knn_seed_leaves > 9 || !(t->knn_seed_leaves & 1) || t->knn_cand < 1 ||
        t->knn_cand > KNN_CAND_MAX || t->order_bits < 8 || t->order_bits > 32 || t->order_bits % 8)
        return PSI_E_ARG;
    ix->knn_tune.seed_leaves = t->knn_seed_leaves;
    ix->knn_tune.cand = t->knn_cand;
    ix->order_bits = t->order_bits;
    return PSI_OK;
}

psi_status psi_get_tuning(psi_index ix, psi_tuning* t) {
    if (!ix || !t) return PSI_E_ARG;
    t->knn_seed_leaves = ix->knn_tune.seed_leaves;
    t->knn_cand = ix->knn_tune.cand;
    t->order_bits = ix->order_bits;
    return PSI_OK;
}

psi_status psi_query_stats(psi_index ix, int enable, uint64_t* h_counts) {
    if (!ix) return PSI_E_ARG;
    psi_status s;
    if (h_counts) {
        if (ix->qstats_on) {
            if ((s = hip_ok(hipStreamSynchronize(ix->st))) != PSI_OK) return s;
            if ((s = hip_ok(hipMemcpy(h_counts, ix->qstats.p, 32, hipMemcpyDeviceToHost))) != PSI_OK) return s;
        } else {
            for (int x = 0; x < 4; ++x) h_counts[x] = 0;
        }
    }
    if (enable && !ix->qstats_on) {
        if (capturing(ix->st)) return PSI_E_STATE;  // allocates
        if ((s = ix->qstats.ensure(32)) != PSI_OK) return s;
        launch_fill_u32(ix->st, ix->qstats.as<uint32_t>(), 8, 0u);
        if ((s = last_launch()) != PSI_OK) return s;
    }
    ix->qstats_on = enable != 0;
    return PSI_OK;
}

psi_status psi_prof_enable(psi_index ix, int on) {
    if (!ix) return PSI_E_ARG;
    ix->prof.on = on != 0;
    return PSI_OK;
}

psi_status psi_prof_only(psi_index ix, const char* family) {
    if (!ix) return PSI_E_ARG;
    ix->prof.only = family ? family : "";
    return PSI_OK;
}

psi_status psi_prof_reset(psi_index ix) {
    if (!ix) return PSI_E_ARG;
    (void)hipStreamSynchronize(ix->st);
    ix->prof.resolve();
    for (auto& kv : ix->prof.fam) {
        kv.second.ms = 0;
        kv.second.launches = 0;
        kv.second.bytes = 0;
    }
    return PSI_OK;
}

psi_status psi_prof_get(psi_index ix, const char* family, double* h_ms, uint64_t* h_launches, uint64_t* h_bytes) {
    if (!ix || !family) return PSI_E_ARG;
    psi_status s = hip_ok(hipStreamSynchronize(ix->st));
    ix->prof.resolve();
    auto it = ix->prof.fam.find(family);
    if (h_ms) *h_ms = it == ix->prof.fam.end() ? 0.0 : it->second.ms;
    if (h_launches) *h_launches = it == ix->prof.fam.end() ? 0 : it->second.launches;
    if (h_bytes) *h_bytes = it == ix->prof.fam.end() ? 0 : it->second.bytes;
    return s;
}

}  // extern "C"
