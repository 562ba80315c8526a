// noalloc_api.cpp -- accumulate_density without device allocation, for callers that
// cannot allocate (code under HIP graph capture, tight serving loops).  Every
// intermediate buffer of the density path (fixation records, spatial-sort keys,
// histogram and scan, sorted points, sorted positions, fixed-point accumulators, maximum,
// counters, the back-face rule's per-point data) lives in one file-scope device array
// of fixed size, laid out for at most
// kMaxPoints points and kMaxFixations fixations.  Each device the library runs on holds
// its own copy until the process ends; its address is taken once per device with
// hipGetSymbolAddress and used from then on (the array's name is not a device address
// in host code).  Calls on one device share that memory: two calls that overlap on one
// device race.  Everything a call reads is written by that call first (accumulators,
// histogram, maximum and counters are cleared by fill kernels at its start).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "gazemap.h"
#include "gm_host.h"
#include "gm_internal.h"

namespace {

constexpr int64_t kMaxPoints = GM_NOALLOC_MAX_POINTS;
constexpr int32_t kMaxFixations = GM_NOALLOC_MAX_FIXATIONS;
constexpr int kMaxDevices = 64;

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// spatial-sort buckets for kMaxPoints points, as density_reserve chooses them
constexpr int64_t max_buckets()
{
    int bits = 1;
    while (bits < 7 && ((int64_t)1 << (3 * bits)) < kMaxPoints) ++bits;
    if (kMaxPoints > ((int64_t)1 << 20)) bits = 8;
    if (kMaxPoints > ((int64_t)1 << 23)) bits = 9;
    return (int64_t)1 << (3 * bits);
}

// scan_tmp_bytes() of the bucket count: one 64-bit partial per scan tile (>= 256
// entries each), so this bounds it
constexpr size_t kScanTmpMax = align256((size_t)(max_buckets() / 256 + 1) * 8);

// the layout, in the order of DensityWork's buffers
constexpr size_t kFixBytes = align256(sizeof(gm::FixRec) * (size_t)kMaxFixations);
constexpr size_t kShiftBytes = 256;
constexpr size_t kKeyBytes = align256(4 * (size_t)kMaxPoints);
constexpr size_t kHistBytes = align256(4 * (size_t)max_buckets());
constexpr size_t kSposBytes = align256(16 * (size_t)kMaxPoints);
constexpr size_t kAccBytes = align256(8 * (size_t)kMaxPoints);
constexpr size_t kStatsBytes = align256(8 * (size_t)gm::kDensityStats);
constexpr size_t kBcandBytes = align256(4 * (size_t)gm::kBfCand * (size_t)kMaxPoints);
constexpr size_t kScratchBytes = kFixBytes + kShiftBytes + kKeyBytes + 2 * kHistBytes + kScanTmpMax + kSposBytes +
                                 2 * kKeyBytes + kAccBytes + 256 + kStatsBytes + kSposBytes + kBcandBytes;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_lock;
void* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device, taken on the first call there.
gm_status scratch_address(int dev, unsigned char*& out)
{
    if (dev < 0 || dev >= kMaxDevices) return gm::fail(GM_ERR_DEVICE, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return gm::fail(GM_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    out = static_cast<unsigned char*>(g_scratch[dev]);
    return GM_OK;
}

// DensityWork whose buffers are ranges of the scratch array
void borrow_work(unsigned char* base, DensityWork& w)
{
    size_t o = 0;
    auto take = [&](gm::DevBuf& b, size_t bytes) {
        b.borrow(base + o, bytes);
        o += bytes;
    };
    take(w.fix, kFixBytes);
    take(w.fx_shift, kShiftBytes);
    take(w.key, kKeyBytes);
    take(w.hist, kHistBytes);
    take(w.cursor, kHistBytes);
    take(w.scan_tmp, kScanTmpMax);
    take(w.spos, kSposBytes);
    take(w.smesh, kKeyBytes);
    take(w.inv, kKeyBytes);
    take(w.acc, kAccBytes);
    take(w.max_acc, 256);
    take(w.stats, kStatsBytes);
    take(w.bface, kSposBytes);
    take(w.bcand, kBcandBytes);
}

}  // namespace

extern "C" gm_status accumulate_density_noalloc(gm_scene* sc, const float* pos, const int32_t* tri,
                                                const int32_t* mesh, int64_t n, const gm_fixations* fix,
                                                double theta_deg, uint32_t flags, float* density,
                                                float* density_norm, float* max_out, void* stream)
{
    gm::clear_error();
    gm_status st = gm::check_density_args(sc, pos, n, fix, theta_deg, flags);
    if (st != GM_OK) return st;
    if (n > kMaxPoints)
        return gm::fail(GM_ERR_CAPACITY, "n = %lld points exceeds the fixed scratch (at most %lld)", (long long)n,
                        (long long)kMaxPoints);
    if (fix->n > kMaxFixations)
        return gm::fail(GM_ERR_CAPACITY, "%d fixations exceed the fixed scratch (at most %d)", fix->n, kMaxFixations);
    if (gm::scan_tmp_bytes(max_buckets()) > kScanTmpMax) return gm::fail(GM_ERR_INTERNAL, "scan scratch too small");
    unsigned char* base = nullptr;
    st = scratch_address(sc->device, base);
    if (st != GM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    DensityWork w;
    borrow_work(base, w);
    st = gm::density_reserve(w, n, fix->n);  // sizes only: every buffer already fits
    if (st != GM_OK) return st;
    gm::DensityLaunch a;
    const int spl = sc->spl ? sc->spl : ((flags & GM_OCC_MASK) != GM_OCC_NONE ? 1 : 2);
    st = gm::density_prep(sc, w, pos, tri, mesh, n, fix, theta_deg, flags & GM_OCC_MASK, spl, 0, a, s);
    if (st != GM_OK) return st;
    if (n > 0 && fix->n > 0) gm::launch_density(a, s);
    return gm::density_finalize(w, n, density, density_norm, max_out, s);
}

extern "C" int64_t gm_noalloc_scratch_bytes(void) { return (int64_t)kScratchBytes; }
