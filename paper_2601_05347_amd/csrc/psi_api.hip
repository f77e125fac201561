// C ABI of the library: index lifetime, build, queries, inspection, timing.
#include <cstring>
#include <new>

#include "psi_index.h"

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

psi_status ensure_q(Buf& b, size_t need, hipStream_t st) {
    if (need <= b.bytes) return PSI_OK;
    if (capturing(st)) return PSI_E_STATE;
    return b.ensure(need);
}

psi_status readback(psi_index ix, const void* dev, size_t bytes) {
    psi_status s = hip_ok(hipMemcpyAsync(ix->pinned, dev, bytes, hipMemcpyDeviceToHost, ix->st));
    if (s != PSI_OK) return s;
    return hip_ok(hipStreamSynchronize(ix->st));
}

// Stable LSD sort of (key, id) pairs; the result lands in sorter.k/i[*which].
// Passes: optionally the four id bytes first (so equal keys end up in id
// order whatever the input order), then the eight key bytes.
psi_status sort_pairs(psi_index ix, const uint64_t* kin, const uint32_t* iin, uint32_t id_base, uint64_t n,
                      bool id_digits, bool hist_ready, int* which, const char* fam, uint32_t key_shift0,
                      int key_passes) {
    Sorter& S = ix->sorter;
    PassList pl{};
    pl.n = 0;
    if (id_digits)
        for (int b = 0; b < 4; ++b) { pl.src[pl.n] = 1; pl.shift[pl.n] = (uint8_t)(8 * b); ++pl.n; }
    for (int b = 0; b < key_passes; ++b) { pl.src[pl.n] = 0; pl.shift[pl.n] = (uint8_t)(key_shift0 + 8 * b); ++pl.n; }
    psi_status s;
    hipStream_t st = ix->st;
    const bool cap = capturing(st);
    if (n <= SORT_SMALL_MAX) {  // every pass in one workgroup's LDS, one launch
        if ((s = ensure_q(S.k[0], std::max<uint64_t>(n, 1) * 8, st)) != PSI_OK) return s;
        if ((s = ensure_q(S.i[0], std::max<uint64_t>(n, 1) * 4, st)) != PSI_OK) return s;
        ProfScope ps(ix, fam, n * 24 * pl.n);
        launch_sort_small(st, kin, iin, id_base, (uint32_t)n, pl, S.k[0].as<uint64_t>(), S.i[0].as<uint32_t>());
        *which = 0;
        return last_launch();
    }
    if ((s = ensure_q(S.hist, MAX_PASSES * RADIX * 4, st)) != PSI_OK) return s;
    if ((s = ensure_q(S.off, MAX_PASSES * RADIX * 4, st)) != PSI_OK) return s;
    if ((s = ensure_q(S.ctr, MAX_PASSES * 4, st)) != PSI_OK) return s;
    for (int b = 0; b < 2; ++b) {
        if ((s = ensure_q(S.k[b], n * 8, st)) != PSI_OK) return s;
        if ((s = ensure_q(S.i[b], n * 4, st)) != PSI_OK) return s;
    }
    const uint64_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
    if (tiles * RADIX > S.status_words) {
        if ((s = ensure_q(S.status, tiles * RADIX * 8, st)) != PSI_OK) return s;
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

// Build sort of n pairs (key, id_base + position), all keys below 2^(top+16):
// two global passes on the key bits [top, top + 16), then every bucket (pairs
// equal in those bits) sorted by its low `top` bits in LDS; buckets too large
// for that take segmented global passes over the low bits. Same result as the
// eight-pass LSD sort: keys ascending, equal keys in id order. Ends with one
// readback (the big-bucket totals); not for graph capture.
constexpr uint64_t BUCKET_MIN_N = 1ull << 24;

// Counts, digit offsets and chunk tables of the two bucket passes, in one
// buffer: cnt [2][XCD_CHUNKS][256] first.
constexpr uint64_t XT_WORDS = 2 * XCD_CHUNKS * RADIX * 2 + XCD_CHUNKS * 4 + XCD_CHUNKS * 8 + 16;

// counted: the chunk counts for these bucket bits are already in the buffer
// (made while encoding). kmax (device, may be null): the largest key, read
// back with the chunk tile counts; if its bucket bits differ from `top`,
// *redo is set, *true_top receives them and nothing is sorted.
psi_status bucket_sort(psi_index ix, const uint64_t* keys, uint32_t id_base, uint64_t n, uint32_t top, bool counted,
                       int* which, const uint64_t* kmax = nullptr, uint32_t* true_top = nullptr,
                       bool* redo = nullptr) {
    Sorter& S = ix->sorter;
    hipStream_t st = ix->st;
    psi_status s;
    if ((s = S.off.ensure(MAX_PASSES * RADIX * 4)) != PSI_OK) return s;
    // tile counters: [0, 8) first pass, [8, 16) second pass, [16, 22) big buckets
    constexpr uint32_t CTR_WORDS = 2 * XCD_CHUNKS + 8;
    if ((s = S.ctr.ensure(CTR_WORDS * 4)) != PSI_OK) return s;
    for (int b = 0; b < 2; ++b) {
        if ((s = S.k[b].ensure(n * 8)) != PSI_OK) return s;
        if ((s = S.i[b].ensure(n * 4)) != PSI_OK) return s;
    }
    auto ensure_status = [&](uint64_t tiles) -> psi_status {
        if (tiles * RADIX <= S.status_words) return PSI_OK;
        psi_status r = S.status.ensure(tiles * RADIX * 8);
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
    const uint32_t nb = BUCKET_COUNT;
    const uint64_t tmpw = scan_tmp_words(nb);
    if ((s = S.bk.ensure(((uint64_t)nb * 5 + 1 + 2 + tmpw) * 4)) != PSI_OK) return s;
    uint32_t* bstart = S.bk.as<uint32_t>();  // nb + 1
    uint32_t* big = bstart + nb + 1;
    uint32_t* ntiles = big + nb;
    uint32_t* tile_off = ntiles + nb;
    uint32_t* big_idx = tile_off + nb;
    uint32_t* totals = big_idx + nb;  // 2
    uint32_t* tmp = totals + 2;
    if (top > 48) return PSI_E_INTERNAL;  // the low bits take at most six 8-bit passes
    // The two bucket passes, each cut into one chunk of consecutive tiles per
    // XCD: per-chunk counts of both digits in one read of the keys, then
    // per-chunk digit offsets and chunk tables (one readback: the tile counts
    // of the second pass's chunks, whose sizes depend on the data).
    const uint64_t T = (n + SORT_TILE - 1) / SORT_TILE;
    if ((s = ensure_status(T + XCD_CHUNKS)) != PSI_OK) return s;
    if ((s = S.xt.ensure(XT_WORDS * 4)) != PSI_OK) return s;
    uint32_t* cnt = S.xt.as<uint32_t>();             // [2][8][256]
    uint32_t* off1 = cnt + 2 * XCD_CHUNKS * RADIX;   // [8][256]
    uint32_t* off2 = off1 + XCD_CHUNKS * RADIX;      // [8][256]
    uint32_t* tw = off2 + XCD_CHUNKS * RADIX;        // first/ntiles of both passes
    uint64_t* tq = reinterpret_cast<uint64_t*>(S.xt.as<char>() + ((reinterpret_cast<char*>(tw + 4 * XCD_CHUNKS) - S.xt.as<char>() + 7) & ~(uint64_t)7));
    ChunkTables tb1{tw, tw + XCD_CHUNKS, tq, tq + XCD_CHUNKS};
    ChunkTables tb2{tw + 2 * XCD_CHUNKS, tw + 3 * XCD_CHUNKS, tq + 2 * XCD_CHUNKS, tq + 3 * XCD_CHUNKS};
    launch_fill_u32(st, S.ctr.as<uint32_t>(), CTR_WORDS, 0u);
    {
        ProfScope ps(ix, "hist", counted ? 0 : n * 8);
        if (!counted) {
            launch_fill_u32(st, cnt, 2 * XCD_CHUNKS * RADIX, 0u);
            launch_hist_chunks(st, keys, n, top, top + 8, cnt);
        }
        launch_chunk_offsets(st, cnt, n, off1, off2, tb1, tb2);
    }
    if ((s = last_launch()) != PSI_OK) return s;
    uint32_t* hq = static_cast<uint32_t*>(ix->pinned);
    if ((s = hip_ok(hipMemcpyAsync(hq, tb2.ntiles, XCD_CHUNKS * 4, hipMemcpyDeviceToHost, st))) != PSI_OK) return s;
    if (kmax && (s = hip_ok(hipMemcpyAsync(hq + XCD_CHUNKS, kmax, 8, hipMemcpyDeviceToHost, st))) != PSI_OK)
        return s;
    if ((s = hip_ok(hipStreamSynchronize(st))) != PSI_OK) return s;
    if (kmax) {
        uint64_t km;
        std::memcpy(&km, hq + XCD_CHUNKS, 8);
        const uint32_t bits = km ? 64u - (uint32_t)__builtin_clzll(km) : 0u;
        *true_top = bits > 16 ? bits - 16 : 0u;
        if (*true_top != top) {
            *redo = true;
            return PSI_OK;
        }
    }
    uint32_t max2 = 0;
    for (uint32_t x = 0; x < XCD_CHUNKS; ++x) max2 = std::max(max2, hq[x]);
    const XcdChunks xc1{tb1.first_tile, tb1.ntiles, tb1.pos_begin, tb1.pos_end};
    const XcdChunks xc2{tb2.first_tile, tb2.ntiles, tb2.pos_begin, tb2.pos_end};
    {
        // 8 B key read (ids implicit), 12 B written
        ProfScope ps(ix, "radix_first", n * 20);
        launch_onesweep_xcd(st, true, keys, nullptr, id_base, S.k[0].as<uint64_t>(), S.i[0].as<uint32_t>(), n, top,
                            off1, S.status.as<uint64_t>(), S.ctr.as<uint32_t>(), next_epoch(), ix->err.as<uint32_t>(),
                            xc1, (uint32_t)((T + XCD_CHUNKS - 1) / XCD_CHUNKS));
    }
    {
        ProfScope ps(ix, "radix_pass", n * 24);
        launch_onesweep_xcd(st, false, S.k[0].as<uint64_t>(), S.i[0].as<uint32_t>(), 0, S.k[1].as<uint64_t>(),
                            S.i[1].as<uint32_t>(), n, top + 8, off2, S.status.as<uint64_t>(),
                            S.ctr.as<uint32_t>() + XCD_CHUNKS, next_epoch(), ix->err.as<uint32_t>(), xc2, max2);
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
    launch_big_tables(st, bstart, big, nb, ntiles, tile_off, big_idx, totals, tmp);
    if ((s = last_launch()) != PSI_OK) return s;
    uint32_t* hp = static_cast<uint32_t*>(ix->pinned);
    if ((s = hip_ok(hipMemcpyAsync(hp, totals, 8, hipMemcpyDeviceToHost, st))) != PSI_OK) return s;
    if ((s = hip_ok(hipMemcpyAsync(hp + 2, ix->err.as<uint32_t>(), 4, hipMemcpyDeviceToHost, st))) != PSI_OK)
        return s;
    if ((s = hip_ok(hipStreamSynchronize(st))) != PSI_OK) return s;
    const uint32_t btiles = hp[0], nbig = hp[1];
    *which = 1;
    // a failed pass is latched in the error word and reported by psi_sync
    if (btiles == 0 || (hp[2] & (ERR_SPIN | ERR_CAPACITY))) return PSI_OK;
    // big buckets: segmented passes over their tiles only (k/i[1] -> [0] -> ... -> [1])
    if (btiles > (n + SORT_TILE - 1) / SORT_TILE + nbig || nbig > nb) return PSI_E_INTERNAL;
    if ((s = ensure_status(btiles)) != PSI_OK) return s;
    const uint64_t seg_words = (uint64_t)btiles * 2 + (uint64_t)nbig * 2;
    if ((s = S.bseg.ensure(seg_words * 4 + (uint64_t)nbig * 8 + 8)) != PSI_OK) return s;
    if ((s = S.shist.ensure((uint64_t)nbig * 8 * RADIX * 4)) != PSI_OK) return s;
    if ((s = S.soff.ensure((uint64_t)nbig * 8 * RADIX * 4)) != PSI_OK) return s;
    uint64_t* seg_begin = S.bseg.as<uint64_t>();
    uint32_t* tile_seg = reinterpret_cast<uint32_t*>(seg_begin + nbig);
    uint32_t* tile_beg = tile_seg + btiles;
    uint32_t* seg_first = tile_beg + btiles;
    uint32_t* seg_end = seg_first + nbig;
    SegTiles sg{tile_seg, tile_beg, seg_first, seg_end, 8 * RADIX};
    // passes over the low bits, an even number so that the result lands in
    // k/i[1] again: an added pass reads bits [8 p, 8 p + 8) inside the
    // bucket bits, constant in a bucket, and changes nothing
    int np = (int)((top + 7) / 8);
    np += np & 1;
    ProfScope ps(ix, "radix_big", (uint64_t)btiles * SORT_TILE * 24 * np);
    launch_big_fill(st, bstart, big, big_idx, tile_off, nb, sg, seg_begin);
    launch_fill_u32(st, S.shist.as<uint32_t>(), (uint64_t)nbig * 8 * RADIX, 0u);
    launch_seg_hist_keys(st, K, btiles, sg, S.shist.as<uint32_t>());
    launch_seg_digit_offsets(st, nbig, S.shist.as<uint32_t>(), seg_begin, S.soff.as<uint32_t>());
    for (int p = 0; p < np; ++p) {
        const int src = (p & 1) ? 0 : 1, dst = 1 - src;
        launch_onesweep(st, false, false, S.k[src].as<uint64_t>(), S.i[src].as<uint32_t>(), 0, S.k[dst].as<uint64_t>(),
                        S.i[dst].as<uint32_t>(), n, 8 * p, S.soff.as<uint32_t>() + p * RADIX, S.status.as<uint64_t>(),
                        S.ctr.as<uint32_t>() + 2 * XCD_CHUNKS + p, next_epoch(), ix->err.as<uint32_t>(), &sg, btiles);
    }
    return last_launch();
}

// Node levels over the current directory: shape on the host, unions on the
// device, from the level just above the leaves up to the root.
psi_status build_nodes(psi_index ix) {
    ix->lv.clear();
    ix->n_inner = 0;
    ix->h = 0;
    if (ix->L == 0) return PSI_OK;
    std::vector<uint64_t> sizes;  // leaves first, root last
    uint64_t n = ix->L;
    sizes.push_back(n);
    while (n > 1) {
        n = (n + ix->B - 1) / ix->B;
        sizes.push_back(n);
    }
    const uint32_t h = (uint32_t)sizes.size() - 1;
    if (h + 1 > (uint32_t)MAX_LEVELS) return PSI_E_INTERNAL;
    ix->h = h;
    ix->lv.resize(h + 1);
    uint64_t off = 0, span = 1;
    for (uint32_t l = 0; l <= h; ++l) {
        ix->lv[l].n = sizes[h - l];
        ix->lv[l].off = l < h ? off : 0;
        if (l < h) off += sizes[h - l];
    }
    for (int l = (int)h; l >= 0; --l) {
        ix->lv[l].span = span;
        span *= ix->B;
    }
    ix->n_inner = off;
    psi_status s = ix->inner.ensure(std::max<uint64_t>(off, 1) * sizeof(NodeRec));
    if (s != PSI_OK) return s;
    // the packed boxes follow on the next kNN (sized here: a captured kNN
    // cannot allocate)
    ix->boxes_fresh = false;
    if ((s = ensure_q(ix->cinner, std::max<uint64_t>(off, 1) * 16, ix->st)) != PSI_OK) return s;
    if ((s = ensure_q(ix->cleaf, std::max<uint64_t>(ix->L, 1) * 16, ix->st)) != PSI_OK) return s;
    NodeRec* inner = ix->inner.as<NodeRec>();
    const NodeRec* leaf = ix->leaf[ix->cur].as<NodeRec>();
    ProfScope ps(ix, "nodes", off * 32 + ix->L * 32);
    for (int l = (int)h - 1; l >= 0; --l) {
        const NodeRec* child = (l + 1 == (int)h) ? leaf : inner + ix->lv[l + 1].off;
        launch_node_level(ix->st, ix->D, child, ix->lv[l + 1].n, inner + ix->lv[l].off, ix->lv[l].n, ix->B,
                          nullptr, nullptr);
    }
    return last_launch();
}

// Curve keys of n points (written to the id table at id_base) and the pairs
// (key, id_base + position) sorted by key, then id, into sorter.k/i[*which]
// (Alg. 3's sort step). Requires n > 0 and the id table sized for them.
psi_status encode_sort(psi_index ix, const uint32_t* d_pts, uint64_t n, uint32_t id_base, int* which) {
    psi_status s;
    Sorter& S = ix->sorter;
    if ((s = S.hist.ensure(MAX_PASSES * RADIX * 4)) != PSI_OK) return s;
    launch_fill_u32(ix->st, S.hist.as<uint32_t>(), 8 * RADIX, 0u);
    uint64_t* keys = ix->idkey.as<uint64_t>() + id_base;
    const bool two_level = ((ix->flags & PSI_FLAG_SORT_BUCKETS) ||
                            (n >= BUCKET_MIN_N && !(ix->flags & PSI_FLAG_SORT_LSD))) &&
                           !capturing(ix->st);
    int w = 0;
    if (two_level) {
        // keys and their maximum; the bucket bits are the 16 below its leading
        // bit. The bucket digits are counted while encoding for a guess of
        // those bits (the previous build's, else the top of the key width);
        // a wrong guess costs one more read of the keys, never a different
        // result.
        if ((s = S.kmax.ensure(8)) != PSI_OK) return s;
        if ((s = S.xt.ensure(XT_WORDS * 4)) != PSI_OK) return s;
        const uint32_t guess = ix->bucket_top <= 48 ? ix->bucket_top : (ix->D == 2 ? 62u : 63u) - 16u;
        launch_fill_u32(ix->st, S.kmax.as<uint32_t>(), 2, 0u);
        launch_fill_u32(ix->st, S.xt.as<uint32_t>(), 2 * XCD_CHUNKS * RADIX, 0u);
        {
            ProfScope ps(ix, "encode_hist", n * (4 * ix->D + 8));
            launch_encode_chunks(ix->st, ix->D, ix->curve, d_pts, n, keys, ix->err.as<uint32_t>(),
                                 S.kmax.as<uint64_t>(), guess, S.xt.as<uint32_t>());
        }
        // the sort starts on the guess; the largest key comes back with the
        // first readback, and a wrong guess redoes the counts
        uint32_t top = guess;
        bool redo = false;
        s = bucket_sort(ix, keys, id_base, n, guess, true, &w, S.kmax.as<uint64_t>(), &top, &redo);
        if (s == PSI_OK && redo) s = bucket_sort(ix, keys, id_base, n, top, false, &w);
        ix->bucket_top = top;
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

// Fresh build of n points whose ids are id_base .. id_base + n - 1 (Alg. 3).
psi_status do_build(psi_index ix, const uint32_t* d_pts, uint64_t n, uint32_t id_base) {
    psi_status s;
    const uint64_t idn = (uint64_t)id_base + n;
    if ((s = ix->idkey.grow_keep(idn * 8, (uint64_t)id_base * 8, ix->st)) != PSI_OK) return s;
    ix->L = 0;
    ix->slot_top = 0;
    ix->n_free = 0;
    if (n == 0) {
        ix->n_live = 0;
        return build_nodes(ix);
    }
    int w = 0;
    if ((s = encode_sort(ix, d_pts, n, id_base, &w)) != PSI_OK) return s;
    Sorter& S = ix->sorter;
    const uint64_t L = (n + ix->phi - 1) / ix->phi;
    const int c = ix->cur;
    if ((s = ix->slots.ensure(L * ix->slot_words() * 4)) != PSI_OK) return s;
    if ((s = ix->leaf[c].ensure(L * sizeof(NodeRec))) != PSI_OK) return s;
    if ((s = ix->pkey[c].ensure(L * 8)) != PSI_OK) return s;
    if ((s = ix->pid[c].ensure(L * 4)) != PSI_OK) return s;
    {
        ProfScope ps(ix, "leaf_fill", n * (12 + 4 * (uint64_t)(ix->D + 1)) + L * 44);
        launch_build_leaves(ix->st, ix->D, ix->curve, S.k[w].as<uint64_t>(), S.i[w].as<uint32_t>(), n, L, ix->C,
                            ix->slots.as<uint32_t>(), ix->pkey[c].as<uint64_t>(), ix->pid[c].as<uint32_t>(),
                            ix->leaf[c].as<NodeRec>());
    }
    ix->L = L;
    ix->slot_top = L;
    ix->n_live = n;
    if ((s = last_launch()) != PSI_OK) return s;
    return build_nodes(ix);
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
    if ((s = ensure_q(ix->scr.c, n * 8, ix->st)) != PSI_OK) return s;
    uint64_t* keys = ix->scr.c.as<uint64_t>();
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
    if ((s = sort_pairs(ix, keys, nullptr, 0, n, false, false, &w, "radix_order", kb - 24, 3)) != PSI_OK) return s;
    *order = ix->sorter.i[w].as<uint32_t>();
    return last_launch();
}

}  // namespace psi

psi::TreeView psi_index_s::view() const {
    psi::TreeView t{};
    t.inner = inner.as<psi::NodeRec>();
    t.leaf = leaf[cur].as<psi::NodeRec>();
    t.cinner = cinner.as<uint4>();
    t.cleaf = cleaf.as<uint4>();
    t.pkey = pkey[cur].as<uint64_t>();
    t.slots = slots.as<uint32_t>();
    t.h = h;
    t.B = B;
    t.C = C;
    t.L = L;
    for (size_t l = 0; l < lv.size() && l < (size_t)psi::MAX_LEVELS; ++l) t.lv[l] = lv[l];
    return t;
}

extern "C" {

const char* psi_status_str(psi_status s) {
    switch (s) {
        case PSI_OK: return "ok";
        case PSI_E_ARG: return "invalid argument";
        case PSI_E_RANGE: return "coordinate out of range";
        case PSI_E_NOMEM: return "out of device memory";
        case PSI_E_CAPACITY: return "id space exhausted";
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
    if (s == PSI_OK) s = hip_ok(hipHostMalloc(&ix->pinned, 4096, hipHostMallocDefault));
    if (s == PSI_OK) s = hip_ok(hipMemsetAsync(ix->err.p, 0, 64, ix->st));
    if (s == PSI_OK) s = hip_ok(hipStreamSynchronize(ix->st));
    if (s != PSI_OK) {
        if (ix->pinned) (void)hipHostFree(ix->pinned);
        delete ix;
        return s;
    }
    *out = ix;
    return PSI_OK;
}

psi_status psi_destroy(psi_index ix) {
    if (!ix) return PSI_E_ARG;
    (void)hipStreamSynchronize(ix->st);
    if (ix->pinned) (void)hipHostFree(ix->pinned);
    delete ix;
    return PSI_OK;
}

psi_status psi_set_stream(psi_index ix, void* hip_stream) {
    if (!ix) return PSI_E_ARG;
    psi_status s = hip_ok(hipStreamSynchronize(ix->st));
    ix->st = static_cast<hipStream_t>(hip_stream);
    return s;
}

psi_status psi_build(psi_index ix, const uint32_t* d_pts, uint64_t n) {
    if (!ix || (n && !d_pts)) return PSI_E_ARG;
    if (capturing(ix->st)) return PSI_E_STATE;
    if (n > 0xFFFFFFFFull) return PSI_E_CAPACITY;
    ix->next_id = 0;
    psi_status s = do_build(ix, d_pts, n, 0);
    if (s == PSI_OK) ix->next_id = (uint32_t)n;
    return s;
}

psi_status psi_batch_insert(psi_index ix, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids) {
    if (!ix || (m && !d_pts)) return PSI_E_ARG;
    if (capturing(ix->st)) return PSI_E_STATE;
    if ((uint64_t)ix->next_id + m > 0xFFFFFFFFull) return PSI_E_CAPACITY;
    if (m == 0) return PSI_OK;
    return do_insert(ix, d_pts, m, d_new_ids);
}

psi_status psi_batch_delete(psi_index ix, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted) {
    if (!ix || (m && !d_ids)) return PSI_E_ARG;
    if (capturing(ix->st)) return PSI_E_STATE;
    if (m > 0xFFFFFFFFull) return PSI_E_ARG;
    return do_delete(ix, d_ids, m, d_ndeleted);
}

psi_status psi_knn(psi_index ix, const uint32_t* d_q, uint64_t nq, uint32_t k, uint32_t* d_ids, uint64_t* d_d2) {
    if (!ix || k == 0 || k > 128 || (nq && (!d_q || !d_ids || !d_d2))) return PSI_E_ARG;
    if (nq == 0) return PSI_OK;
    const uint32_t* order = nullptr;
    psi_status s = query_order(ix, d_q, nq, false, &order);
    if (s != PSI_OK) return s;
    // The box tests read the packed boxes: rewritten after the tree changed,
    // and always inside a captured graph (a replay may follow updates).
    const bool cap = capturing(ix->st);
    if (ix->L && (!ix->boxes_fresh || cap)) {
        if ((s = ensure_q(ix->cinner, std::max<uint64_t>(ix->n_inner, 1) * 16, ix->st)) != PSI_OK) return s;
        if ((s = ensure_q(ix->cleaf, ix->L * 16, ix->st)) != PSI_OK) return s;
        ProfScope pb(ix, "pack_boxes", (ix->n_inner + ix->L) * 48);
        launch_pack_boxes(ix->st, ix->D, ix->leaf[ix->cur].as<NodeRec>(), ix->L, ix->cleaf.as<uint4>());
        launch_pack_boxes(ix->st, ix->D, ix->inner.as<NodeRec>(), ix->n_inner, ix->cinner.as<uint4>());
        if (!cap) ix->boxes_fresh = true;
    }
    ProfScope ps(ix, "knn", nq * (4ull * ix->D + 12ull * k));
    launch_knn(ix->st, ix->D, ix->view(), d_q, ix->scr.c.as<uint64_t>(), nq, order, k,
               (ix->flags & PSI_FLAG_KNN_NEAREST_FIRST) ? 1 : 0, d_ids, d_d2);
    return last_launch();
}

psi_status psi_range_count(psi_index ix, const uint32_t* d_boxes, uint64_t nb, uint64_t* d_counts) {
    if (!ix || (nb && (!d_boxes || !d_counts))) return PSI_E_ARG;
    if (nb == 0) return PSI_OK;
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
    const uint32_t* order = nullptr;
    psi_status s = query_order(ix, d_boxes, nb, true, &order);
    if (s != PSI_OK) return s;
    ProfScope ps(ix, "range_report", nb * (8ull * ix->D + 16));
    launch_range_report(ix->st, ix->D, ix->view(), d_boxes, nb, order, d_offsets, d_ids);
    return last_launch();
}

psi_status psi_sync(psi_index ix) {
    if (!ix) return PSI_E_ARG;
    psi_status s = readback(ix, ix->err.p, 4);
    if (s != PSI_OK) return s;
    uint32_t e = 0;
    std::memcpy(&e, ix->pinned, 4);
    if (e) {
        (void)hipMemsetAsync(ix->err.p, 0, 4, ix->st);
        (void)hipStreamSynchronize(ix->st);
        if (e & ERR_RANGE) return PSI_E_RANGE;
        return PSI_E_INTERNAL;
    }
    return PSI_OK;
}

psi_status psi_size(psi_index ix, uint64_t* h_n_live) {
    if (!ix || !h_n_live) return PSI_E_ARG;
    psi_status s = psi_sync(ix);
    *h_n_live = ix->n_live;
    return s;
}

psi_status psi_next_id(psi_index ix, uint32_t* h_next_id) {
    if (!ix || !h_next_id) return PSI_E_ARG;
    *h_next_id = ix->next_id;
    return PSI_OK;
}

psi_status psi_export(psi_index ix, uint64_t* d_keys, uint32_t* d_ids, uint32_t* d_pts) {
    if (!ix) return PSI_E_ARG;
    if (ix->L == 0) return PSI_OK;
    psi_status s;
    if ((s = ix->scr.a.ensure((ix->L + 1) * 8)) != PSI_OK) return s;
    if ((s = ix->scr.b.ensure((2 * ix->L + scan_tmp_words(ix->L) + 4) * 8)) != PSI_OK) return s;
    launch_leaf_offsets(ix->st, ix->leaf[ix->cur].as<NodeRec>(), ix->L, ix->scr.a.as<uint64_t>(), ix->scr.b.as<uint64_t>());
    launch_export_sorted(ix->st, ix->D, ix->curve, ix->view(), ix->scr.a.as<uint64_t>(), d_keys, d_ids, d_pts);
    return last_launch();
}

psi_status psi_export_leaves(psi_index ix, uint32_t* d_ids, uint32_t* d_pts) {
    if (!ix) return PSI_E_ARG;
    if (ix->L == 0) return PSI_OK;
    psi_status s;
    if ((s = ix->scr.a.ensure((ix->L + 1) * 8)) != PSI_OK) return s;
    if ((s = ix->scr.b.ensure((2 * ix->L + scan_tmp_words(ix->L) + 4) * 8)) != PSI_OK) return s;
    launch_leaf_offsets(ix->st, ix->leaf[ix->cur].as<NodeRec>(), ix->L, ix->scr.a.as<uint64_t>(), ix->scr.b.as<uint64_t>());
    launch_export_raw(ix->st, ix->D, ix->view(), ix->scr.a.as<uint64_t>(), d_ids, d_pts);
    return last_launch();
}

psi_status psi_shape(psi_index ix, uint64_t* h_n_leaves, uint32_t* h_height, uint64_t* h_level_sizes) {
    if (!ix || !h_n_leaves || !h_height) return PSI_E_ARG;
    *h_n_leaves = ix->L;
    *h_height = ix->h;
    if (h_level_sizes)
        for (uint32_t l = 0; l < ix->lv.size(); ++l) h_level_sizes[l] = ix->lv[l].n;
    return PSI_OK;
}

psi_status psi_export_structure(psi_index ix, uint64_t* d_piv_key, uint32_t* d_piv_id, uint32_t* d_leaf_cnt,
                                uint32_t* d_leaf_lo, uint32_t* d_leaf_hi, uint32_t* d_node_lo, uint32_t* d_node_hi,
                                uint64_t* d_node_cnt) {
    if (!ix) return PSI_E_ARG;
    launch_export_structure(ix->st, ix->D, ix->view(), ix->n_inner, ix->pkey[ix->cur].as<uint64_t>(),
                            ix->pid[ix->cur].as<uint32_t>(), d_piv_key, d_piv_id, d_leaf_cnt, d_leaf_lo, d_leaf_hi,
                            d_node_lo, d_node_hi, d_node_cnt);
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
};

psi_status psi_graph_begin(void* hip_stream) {
    return hip_ok(hipStreamBeginCapture(static_cast<hipStream_t>(hip_stream), hipStreamCaptureModeThreadLocal));
}

psi_status psi_graph_end(void* hip_stream, psi_graph* out) {
    if (!out) return PSI_E_ARG;
    *out = nullptr;
    psi_graph g = new (std::nothrow) psi_graph_s;
    hipGraph_t graph = nullptr;
    psi_status s = hip_ok(hipStreamEndCapture(static_cast<hipStream_t>(hip_stream), &graph));
    if (!g) {
        if (graph) (void)hipGraphDestroy(graph);
        return PSI_E_NOMEM;
    }
    if (s == PSI_OK) s = hip_ok(hipGraphInstantiate(&g->e, graph, nullptr, nullptr, 0));
    g->g = graph;
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
    return hip_ok(hipGraphLaunch(g->e, static_cast<hipStream_t>(hip_stream)));
}

psi_status psi_graph_destroy(psi_graph g) {
    if (!g) return PSI_E_ARG;
    if (g->e) (void)hipGraphExecDestroy(g->e);
    if (g->g) (void)hipGraphDestroy(g->g);
    delete g;
    return PSI_OK;
}

psi_status psi_prof_enable(psi_index ix, int on) {
    if (!ix) return PSI_E_ARG;
    ix->prof.on = on != 0;
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
