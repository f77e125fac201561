// psi_sort_pairs_noalloc: the (key, id) sort of psi_sort_pairs without any
// allocation, for callers that cannot allocate (graph capture, serving loops
// that must not call the allocator). Its workspace is one file-scope device
// array, `scratch`, of fixed size; every GPU the library runs on holds its
// own copy until the process ends. Host code never passes the array's name
// to a kernel (on the host that name is only a stand-in, not a device
// address): the first call on a device looks up the array's device address
// with hipGetSymbolAddress, with that device current, and keeps it per
// device; kernels receive that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/psi.h"
#include "psi_kern.h"

namespace psi {
namespace {

constexpr uint64_t NA_MAX = PSI_SORT_NOALLOC_MAX;        // pairs
constexpr uint64_t NA_TILES = (NA_MAX + SORT_TILE - 1) / SORT_TILE;
constexpr int NA_PASSES = 12;                            // four id bytes, then eight key bytes
// Layout of the workspace (byte offsets, each 256-aligned).
constexpr uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }
constexpr uint64_t OFF_K0 = 0;
constexpr uint64_t OFF_K1 = OFF_K0 + align256(NA_MAX * 8);
constexpr uint64_t OFF_I0 = OFF_K1 + align256(NA_MAX * 8);
constexpr uint64_t OFF_I1 = OFF_I0 + align256(NA_MAX * 4);
constexpr uint64_t OFF_HIST = OFF_I1 + align256(NA_MAX * 4);
constexpr uint64_t OFF_DOFF = OFF_HIST + align256(NA_PASSES * RADIX * 4);
constexpr uint64_t OFF_CTR = OFF_DOFF + align256(NA_PASSES * RADIX * 4);
constexpr uint64_t OFF_ERR = OFF_CTR + align256(NA_PASSES * 4);
constexpr uint64_t OFF_STATUS = OFF_ERR + 256;
constexpr uint64_t NA_BYTES = OFF_STATUS + align256(NA_TILES * RADIX * 8);

}  // namespace
}  // namespace psi

// The workspace (about 25 MB at the maximum of 2^20 pairs).
static __device__ __align__(256) unsigned char scratch[psi::NA_BYTES];

namespace psi {
namespace {

struct DeviceScratch {
    unsigned char* ptr = nullptr;  // device address of `scratch` on this device
    uint32_t epoch = 0;            // look-back epochs used so far on this device
};
std::mutex na_mu;
DeviceScratch na_dev[64];

// The workspace of the current device: its address looked up once (status
// words cleared with a kernel at that point), and the next look-back epochs.
psi_status na_workspace(hipStream_t st, unsigned char** base, uint32_t* epoch0, int passes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return PSI_E_HIP;
    }
    std::lock_guard<std::mutex> lk(na_mu);
    DeviceScratch& d = na_dev[dev];
    if (!d.ptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return PSI_E_HIP;
        }
        d.ptr = static_cast<unsigned char*>(p);
        launch_fill_u32(st, reinterpret_cast<uint32_t*>(d.ptr + OFF_STATUS), NA_TILES * RADIX * 2, 0u);
        d.epoch = 0;
    }
    if (d.epoch + passes >= (1u << 30)) {
        launch_fill_u32(st, reinterpret_cast<uint32_t*>(d.ptr + OFF_STATUS), NA_TILES * RADIX * 2, 0u);
        d.epoch = 0;
    }
    *epoch0 = d.epoch + 1;
    d.epoch += passes;
    *base = d.ptr;
    return PSI_OK;
}

bool na_capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return cs == hipStreamCaptureStatusActive;
}

}  // namespace
}  // namespace psi

extern "C" psi_status psi_sort_pairs_noalloc(const uint64_t* d_keys, const uint32_t* d_ids, uint64_t n,
                                             uint64_t* d_keys_out, uint32_t* d_ids_out, void* hip_stream) {
    using namespace psi;
    if (n && (!d_keys || !d_ids || !d_keys_out || !d_ids_out)) return PSI_E_ARG;
    if (n > NA_MAX) return PSI_E_ARG;
    if (n == 0) return PSI_OK;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    PassList pl{};
    pl.n = 0;
    for (int b = 0; b < 4; ++b) { pl.src[pl.n] = 1; pl.shift[pl.n] = (uint8_t)(8 * b); ++pl.n; }
    for (int b = 0; b < 8; ++b) { pl.src[pl.n] = 0; pl.shift[pl.n] = (uint8_t)(8 * b); ++pl.n; }
    if (n <= SORT_SMALL_MAX) {  // one workgroup, every pass in LDS, straight into the outputs
        launch_sort_small(st, d_keys, d_ids, 0, (uint32_t)n, pl, d_keys_out, d_ids_out);
        return hipGetLastError() == hipSuccess ? PSI_OK : PSI_E_HIP;
    }
    unsigned char* base = nullptr;
    uint32_t epoch = 0;
    psi_status s = na_workspace(st, &base, &epoch, pl.n);
    if (s != PSI_OK) return s;
    uint64_t* K[2] = {reinterpret_cast<uint64_t*>(base + OFF_K0), reinterpret_cast<uint64_t*>(base + OFF_K1)};
    uint32_t* I[2] = {reinterpret_cast<uint32_t*>(base + OFF_I0), reinterpret_cast<uint32_t*>(base + OFF_I1)};
    uint32_t* hist = reinterpret_cast<uint32_t*>(base + OFF_HIST);
    uint32_t* doff = reinterpret_cast<uint32_t*>(base + OFF_DOFF);
    uint32_t* ctr = reinterpret_cast<uint32_t*>(base + OFF_CTR);
    uint32_t* err = reinterpret_cast<uint32_t*>(base + OFF_ERR);
    uint64_t* status = reinterpret_cast<uint64_t*>(base + OFF_STATUS);
    const uint64_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
    const bool cap = na_capturing(st);
    // what every call must find zeroed: histograms and tile counters (the
    // status words carry an epoch instead; a captured graph replays its
    // epochs, so under capture they are cleared before each pass)
    launch_fill_u32(st, hist, (uint64_t)pl.n * RADIX, 0u);
    launch_fill_u32(st, ctr, NA_PASSES, 0u);
    launch_hist_pairs(st, d_keys, d_ids, 0, n, pl, hist);
    launch_digit_offsets(st, pl.n, hist, doff);
    const uint64_t* ksrc = d_keys;
    const uint32_t* isrc = d_ids;
    for (int p = 0; p < pl.n; ++p) {
        const bool last = p + 1 == pl.n;
        uint64_t* kd = last ? d_keys_out : K[p & 1];
        uint32_t* id = last ? d_ids_out : I[p & 1];
        if (cap) launch_fill_u32(st, reinterpret_cast<uint32_t*>(status), tiles * RADIX * 2, 0u);
        launch_onesweep(st, false, pl.src[p] == 1, ksrc, isrc, 0, kd, id, n, pl.shift[p], doff + p * RADIX, status,
                        ctr + p, epoch + (uint32_t)p, err);
        ksrc = kd;
        isrc = id;
    }
    return hipGetLastError() == hipSuccess ? PSI_OK : PSI_E_HIP;
}
