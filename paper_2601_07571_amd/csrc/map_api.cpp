// map_api.cpp -- incremental density maps (include/gazemap.h, gm_map_*): a fixed set
// of points, sorted once, whose fixed-point accumulators take fixations in blocks,
// each block filtered by a start-time window and charged to a duration budget.
// rho is linear in the fixations (Sec. 3.2.1 sums one term per fixation), so
// adding blocks one after the other gives exactly the map of their union.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gazemap.h"
#include "gm_host.h"
#include "gm_internal.h"

using namespace gm;

namespace {

// counters[]: budget used, budget total (units of 2^-10 s), fixations added,
// invalid, over budget
constexpr int kMapCounters = 5;
constexpr double kBudgetUnit = 1024.0;  // units per second
// Blocks of a plain map are gathered: their selected fixation records are appended to
// one buffer, and one density launch takes them all (at the next read, or when this
// many fixations are pending).  A launch per block left the GPU idle in each launch's
// tail; the sum is the same bit for bit (fixed-point accumulation).
constexpr int64_t kPendingMax = 65536;

}  // namespace

struct gm_map {
    gm_scene* scene = nullptr;
    int device = 0;
    int64_t n = 0;
    double sigma = 0.0;
    uint32_t mode = 0;
    int spl = 1;
    int32_t shift = 0;
    unsigned long long budget_units = 0;
    DensityWork w;     // sorted points, accumulators, records of the last block
    DevBuf live;       // records taken so far (pending blocks) / of the block being added
    DevBuf pending;    // plain maps: records of the blocks not yet accumulated [kPendingMax]
    int64_t pending_hi = 0;  // upper bound of the pending records (sum of the blocks' sizes)
    DevBuf counters;   // [kMapCounters] uint64
    // posed maps: points grouped by mesh, mesh m at sorted entries [moff[m], moff[m + 1]);
    // per block, records [M][stride] and pose pairs [M][stride][24]
    bool posed = false;
    std::vector<int64_t> moff;
    DevBuf recs, xf;
    // recorded on the stream of every add whose records are pending: the next add (on any
    // stream) and the gathered launch wait for it, so pending blocks are complete whichever
    // streams queued them
    hipEvent_t added = nullptr;
    ~gm_map()
    {
        if (added) (void)hipEventDestroy(added);
    }
};

namespace gm {

// One BVH per mesh in the mesh's own frame, from the scene's triangle records (the
// same FP32 vertices), with the octant node copies and axis-permuted record copies of
// the scene BVH; record ids stay scene-global.
gm_status ensure_blas(gm_scene* sc)
{
    if (!sc->blas.empty()) return GM_OK;
    const int32_t M = sc->M;
    std::vector<std::vector<int64_t>> per((size_t)M);
    for (size_t i = 0; i < sc->bvh.tris.size(); ++i) {
        const BvhTri& r = sc->bvh.tris[i];
        if (r.id >= 0 && r.mesh >= 0 && r.mesh < M) per[(size_t)r.mesh].push_back((int64_t)i);
    }
    std::vector<BvhNode> all_nodes;
    std::vector<BvhTri> all_tris;
    std::vector<BlasDesc> desc((size_t)M);
    for (int32_t m = 0; m < M; ++m) {
        const std::vector<int64_t>& ids = per[(size_t)m];
        const int64_t Tm = (int64_t)ids.size();
        std::vector<float> V((size_t)(9 * std::max<int64_t>(Tm, 1)));
        std::vector<int32_t> I((size_t)(3 * std::max<int64_t>(Tm, 1))), tm((size_t)std::max<int64_t>(Tm, 1), m),
            gid((size_t)std::max<int64_t>(Tm, 1));
        for (int64_t j = 0; j < Tm; ++j) {
            const BvhTri& r = sc->bvh.tris[(size_t)ids[(size_t)j]];
            for (int k = 0; k < 3; ++k) {
                V[(size_t)(9 * j + k)] = r.v0[k];
                V[(size_t)(9 * j + 3 + k)] = r.v1[k];
                V[(size_t)(9 * j + 6 + k)] = r.v2[k];
                I[(size_t)(3 * j + k)] = (int32_t)(3 * j + k);
            }
            gid[(size_t)j] = r.id;
        }
        HostBvh hb;
        build_bvh(V.data(), I.data(), tm.data(), Tm, hb);
        for (BvhTri& r : hb.tris)
            if (r.id >= 0) r.id = gid[(size_t)r.id];
        std::vector<BvhNode> n8;
        octant_node_copies(hb.nodes, n8);
        std::vector<BvhTri> t3;
        permute_tri_copies(hb.tris, t3);
        desc[(size_t)m] = BlasDesc{(int64_t)all_nodes.size(), (int64_t)hb.nodes.size(), (int64_t)all_tris.size(),
                                   (int64_t)hb.tris.size()};
        all_nodes.insert(all_nodes.end(), n8.begin(), n8.end());
        all_tris.insert(all_tris.end(), t3.begin(), t3.end());
    }
    auto up = [&](DevBuf& b, const void* src, size_t bytes) -> hipError_t {
        hipError_t e = b.ensure(bytes);
        if (e != hipSuccess) return e;
        return hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice);
    };
    hipError_t e = up(sc->blas_nodes, all_nodes.data(), all_nodes.size() * sizeof(BvhNode));
    if (e == hipSuccess) e = up(sc->blas_tris, all_tris.data(), all_tris.size() * sizeof(BvhTri));
    if (e == hipSuccess) e = up(sc->blas_desc, desc.data(), desc.size() * sizeof(BlasDesc));
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? GM_ERR_OUT_OF_MEMORY : GM_ERR_DEVICE, "per-mesh BVH upload: %s",
                    hipGetErrorString(e));
    sc->blas = desc;
    return GM_OK;
}

}  // namespace gm

namespace {

gm_status check_map(const gm_map* m)
{
    if (!m) return fail(GM_ERR_INVALID_ARGUMENT, "map is NULL");
    int dev = -1;
    GM_HIP(hipGetDevice(&dev));
    if (dev != m->device)
        return fail(GM_ERR_INVALID_ARGUMENT, "map lives on device %d but device %d is current", m->device, dev);
    return GM_OK;
}

// one density launch over the pending records of a plain map
gm_status map_flush(gm_map* m, hipStream_t s)
{
    if (m->pending_hi == 0) return GM_OK;
    GM_HIP(hipStreamWaitEvent(s, m->added, 0));
    if (m->n > 0) {
        DensityLaunch a;
        density_args(m->scene, m->w, m->n, (int32_t)m->pending_hi, m->sigma, m->mode, m->spl, 0, a);
        a.fix = m->pending.as<FixRec>();
        a.F_live = m->live.as<unsigned int>();
        zero(m->w.stats.p, 8 * kDensityStats, s);
        launch_density(a, s);
    }
    zero(m->live.p, 4, s);
    m->pending_hi = 0;
    GM_HIP(hipGetLastError());
    return GM_OK;
}

// accumulators, maximum and counters back to zero; the budget total set again
gm_status map_clear(gm_map* m, hipStream_t s)
{
    zero(m->live.p, 4, s);  // pending blocks are dropped with the rest
    m->pending_hi = 0;
    if (m->n > 0) zero(m->w.acc.p, 8 * (size_t)m->n, s);
    zero(m->counters.p, 8 * kMapCounters, s);
    const unsigned long long b = m->budget_units;  // counters[1], as two little-endian words
    fill_u32(static_cast<uint32_t*>(m->counters.p) + 2, 1, (uint32_t)(b & 0xFFFFFFFFull), s);
    fill_u32(static_cast<uint32_t*>(m->counters.p) + 3, 1, (uint32_t)(b >> 32), s);
    GM_HIP(hipGetLastError());
    return GM_OK;
}

gm_status check_block(const gm_map* m, const gm_fixations* fix, const double* time, double t_begin, double t_end)
{
    gm_status st = check_map(m);
    if (st != GM_OK) return st;
    if (!fix) return fail(GM_ERR_INVALID_ARGUMENT, "fixations is NULL");
    if (fix->n < 0) return fail(GM_ERR_INVALID_ARGUMENT, "fixation count < 0");
    if (fix->n > 0 && (!fix->eye || !fix->gaze || !fix->duration))
        return fail(GM_ERR_INVALID_ARGUMENT, "fixation arrays must not be NULL");
    if (time && (std::isnan(t_begin) || std::isnan(t_end)))
        return fail(GM_ERR_INVALID_ARGUMENT, "the time window bounds must not be NaN");
    return GM_OK;
}

}  // namespace

extern "C" {

gm_status gm_map_create(gm_scene* sc, const float* pos, const int32_t* tri, const int32_t* mesh, int64_t n,
                        double theta_deg, uint32_t flags, double max_total_duration, gm_map** out, void* stream)
{
    clear_error();
    if (!out) return fail(GM_ERR_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    if (!sc) return fail(GM_ERR_INVALID_ARGUMENT, "scene is NULL");
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GM_ERR_INVALID_ARGUMENT, "n must be in [0, 2^31)");
    if (n > 0 && !pos) return fail(GM_ERR_INVALID_ARGUMENT, "pos is NULL");
    if (!(theta_deg > 0.0 && theta_deg < 45.0)) return fail(GM_ERR_INVALID_ARGUMENT, "theta_deg must be in (0, 45)");
    const uint32_t mode = flags & GM_OCC_MASK;
    const bool posed = (flags & GM_MAP_POSED) != 0;
    if (mode > GM_OCC_FULL || (flags & ~(GM_OCC_MASK | GM_MAP_POSED)))
        return fail(GM_ERR_INVALID_ARGUMENT, "unknown flags 0x%x", flags);
    if (posed && n > 0 && !mesh) return fail(GM_ERR_INVALID_ARGUMENT, "a posed map needs the points' mesh ids");
    if (!(max_total_duration > 0.0 && max_total_duration <= 1e9))
        return fail(GM_ERR_INVALID_ARGUMENT, "max_total_duration must be in (0, 1e9] seconds");
    gm_status st = check_device(sc);
    if (st != GM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> moff;
    if (posed) {
        // points must come grouped by mesh (as the samplers write them)
        std::vector<int32_t> hm((size_t)std::max<int64_t>(n, 1));
        if (n > 0) {
            GM_HIP(hipStreamSynchronize(s));
            GM_HIP(hipMemcpy(hm.data(), mesh, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
        }
        moff.assign((size_t)sc->M + 1, 0);
        for (int64_t i = 0; i < n; ++i) {
            const int32_t v = hm[(size_t)i];
            if (v < 0 || v >= sc->M) return fail(GM_ERR_INVALID_ARGUMENT, "point %lld: mesh %d out of range", (long long)i, v);
            if (i > 0 && v < hm[(size_t)i - 1])
                return fail(GM_ERR_INVALID_ARGUMENT, "a posed map needs its points grouped by mesh, in mesh order");
            ++moff[(size_t)v + 1];
        }
        for (int32_t k = 0; k < sc->M; ++k) moff[(size_t)k + 1] += moff[(size_t)k];
        if (mode != GM_OCC_NONE) {
            st = ensure_blas(sc);
            if (st != GM_OK) return st;
        }
    }

    gm_map* m = new gm_map;
    {
        const hipError_t e = hipEventCreateWithFlags(&m->added, hipEventDisableTiming);
        if (e != hipSuccess) {
            m->added = nullptr;
            delete m;
            return fail(GM_ERR_DEVICE, "hipEventCreateWithFlags: %s", hipGetErrorString(e));
        }
    }
    m->posed = posed;
    m->moff = moff;
    m->scene = sc;
    m->device = sc->device;
    m->n = n;
    m->sigma = std::tan(theta_deg * M_PI / 180.0);
    m->mode = mode;
    m->spl = sc->spl ? sc->spl : (mode != GM_OCC_NONE ? 1 : 2);
    m->budget_units = (unsigned long long)std::floor(max_total_duration * kBudgetUnit);
    // rho_s <= sum of the weights t / (sigma sqrt(2 pi)) of the fixations taken <= D / (sigma sqrt(2 pi))
    int e = 0;
    (void)std::frexp(2.0 * max_total_duration / (m->sigma * std::sqrt(2.0 * M_PI)), &e);
    m->shift = 62 - e;
    st = density_reserve(m->w, n, 1);
    if (st == GM_OK && m->live.ensure(16) != hipSuccess) st = fail(GM_ERR_OUT_OF_MEMORY, "map counters");
    if (st == GM_OK && m->counters.ensure(8 * kMapCounters) != hipSuccess)
        st = fail(GM_ERR_OUT_OF_MEMORY, "map counters");
    if (st != GM_OK) {
        delete m;
        return st;
    }
    fill_u32(m->w.fx_shift.p, 1, (uint32_t)m->shift, s);
    if (!posed) {
        density_sort(sc, m->w, pos, tri, mesh, n, s);
        st = density_backface(sc, m->w, n, m->mode, s);
        if (st != GM_OK) {
            delete m;
            return st;
        }
    } else {
        for (int32_t k = 0; k < sc->M; ++k) {
            const int64_t off = moff[(size_t)k], nk = moff[(size_t)k + 1] - off;
            density_sort(sc, m->w, pos + 3 * off, tri ? tri + off : nullptr, mesh + off, nk, s, off);
        }
        // The back-face rule per mesh segment, in the meshes' own frames: a launch for mesh
        // k sees its samples and the fixations in k's frame, where the rule's closedness,
        // box and neighbour data hold for every pose (the motion is rigid).  The buffers
        // are sized for all points first (a segment call must not reallocate them).
        if (m->mode != GM_OCC_NONE && sc->any_closed() && n > 0) {
            st = (m->w.bface.ensure(16 * (size_t)n) == hipSuccess &&
                  m->w.bcand.ensure(4 * (size_t)kBfCand * (size_t)n) == hipSuccess)
                     ? GM_OK
                     : fail(GM_ERR_OUT_OF_MEMORY, "back-face rule data");
            bool all = true;
            for (int32_t k = 0; k < sc->M && st == GM_OK; ++k) {
                const int64_t off = moff[(size_t)k], nk = moff[(size_t)k + 1] - off;
                if (nk <= 0) continue;
                st = density_backface(sc, m->w, nk, m->mode, s, off);
                all = all && m->w.backface;
            }
            m->w.backface = st == GM_OK && all;
            if (st != GM_OK) {
                delete m;
                return st;
            }
        }
    }
    st = map_clear(m, s);
    if (st == GM_OK) {
        const hipError_t e2 = hipGetLastError();
        if (e2 != hipSuccess) st = fail(GM_ERR_DEVICE, "map create: %s", hipGetErrorString(e2));
    }
    if (st != GM_OK) {
        delete m;
        return st;
    }
    *out = m;
    return GM_OK;
}

gm_status gm_map_add(gm_map* m, const gm_fixations* fix, const double* time, double t_begin, double t_end,
                     void* stream)
{
    clear_error();
    gm_status st = check_block(m, fix, time, t_begin, t_end);
    if (st != GM_OK) return st;
    if (m->posed) return fail(GM_ERR_INVALID_ARGUMENT, "a posed map takes its fixations with gm_map_add_posed");
    hipStream_t s = (hipStream_t)stream;
    const int32_t F = fix->n;
    if (F == 0) return GM_OK;
    unsigned long long* c = m->counters.as<unsigned long long>();
    if (F > kPendingMax) {
        // a large block: the pending ones first, then this one in a launch of its own
        st = map_flush(m, s);
        if (st != GM_OK) return st;
        GM_HIP(m->w.fix.ensure(sizeof(FixRec) * (size_t)F));
        launch_fix_select(fix->eye, fix->gaze, fix->duration, time, F, t_begin, t_end, m->sigma, kGateWiden,
                          m->w.fix.as<FixRec>(), m->live.as<unsigned int>(), c, c + 2, s);
        if (m->n > 0) {
            DensityLaunch a;
            density_args(m->scene, m->w, m->n, F, m->sigma, m->mode, m->spl, 0, a);
            a.F_live = m->live.as<unsigned int>();
            zero(m->w.stats.p, 8 * kDensityStats, s);
            launch_density(a, s);
        }
        zero(m->live.p, 4, s);
        GM_HIP(hipGetLastError());
        return GM_OK;
    }
    if (m->pending_hi + F > kPendingMax) {
        st = map_flush(m, s);
        if (st != GM_OK) return st;
    }
    // allocated once (nothing pending can be lost by a reallocation)
    GM_HIP(m->pending.ensure(sizeof(FixRec) * (size_t)kPendingMax));
    if (m->pending_hi > 0) GM_HIP(hipStreamWaitEvent(s, m->added, 0));  // after the pending adds
    launch_fix_select(fix->eye, fix->gaze, fix->duration, time, F, t_begin, t_end, m->sigma, kGateWiden,
                      m->pending.as<FixRec>(), m->live.as<unsigned int>(), c, c + 2, s);
    m->pending_hi += F;
    GM_HIP(hipGetLastError());
    GM_HIP(hipEventRecord(m->added, s));
    return GM_OK;
}

gm_status gm_map_add_posed(gm_map* m, const gm_fixations* fix, const float* pose, const double* time,
                           double t_begin, double t_end, void* stream)
{
    clear_error();
    gm_status st = check_block(m, fix, time, t_begin, t_end);
    if (st != GM_OK) return st;
    if (!m->posed) return fail(GM_ERR_INVALID_ARGUMENT, "the map was not created with GM_MAP_POSED");
    const int32_t F = fix->n;
    if (F > 0 && !pose) return fail(GM_ERR_INVALID_ARGUMENT, "pose is NULL");
    if (F == 0) return GM_OK;
    hipStream_t s = (hipStream_t)stream;
    gm_scene* sc = m->scene;
    const int32_t M = sc->M;
    const int64_t stride = F;
    GM_HIP(m->recs.ensure(sizeof(FixRec) * (size_t)M * (size_t)stride));
    GM_HIP(m->xf.ensure(sizeof(float) * 24 * (size_t)M * (size_t)stride));
    unsigned long long* c = m->counters.as<unsigned long long>();
    zero(m->live.p, 4, s);
    launch_fix_posed(fix->eye, fix->gaze, fix->duration, time, pose, F, M, stride, t_begin, t_end, m->sigma,
                     kGateWiden, m->recs.as<FixRec>(), m->xf.as<float>(), m->live.as<unsigned int>(), c, c + 2, s);
    zero(m->w.stats.p, 8 * kDensityStats, s);
    for (int32_t k = 0; k < M; ++k) {
        const int64_t off = m->moff[(size_t)k], nk = m->moff[(size_t)k + 1] - off;
        if (nk <= 0) continue;
        DensityLaunch a;
        density_args(sc, m->w, nk, F, m->sigma, m->mode, m->spl, 0, a);
        a.spos += off;
        a.smesh += off;
        a.acc += off;
        a.fix = m->recs.as<FixRec>() + (int64_t)k * stride;
        a.F_live = m->live.as<unsigned int>();
        if (a.bface) {
            a.bface += off;
            a.bcand += kBfCand * off;
        }
        if (m->mode != GM_OCC_NONE) {
            a.blas = sc->blas_desc.as<BlasDesc>();
            a.blas_nodes = sc->blas_nodes.as<BvhNode>();
            a.blas_tris = sc->blas_tris.as<BvhTri>();
            a.fix_all = m->recs.as<FixRec>();
            a.xf = m->xf.as<float>();
            a.fix_stride = stride;
            a.n_inst = M;
            a.self_mesh = k;
        }
        launch_density(a, s);
    }
    GM_HIP(hipGetLastError());
    return GM_OK;
}

gm_status gm_map_read(gm_map* m, float* density, float* density_norm, float* max_out, void* stream)
{
    clear_error();
    gm_status st = check_map(m);
    if (st != GM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    st = map_flush(m, s);
    if (st != GM_OK) return st;
    zero(m->w.max_acc.p, 8, s);
    return density_finalize(m->w, m->n, density, density_norm, max_out, s);
}

gm_status gm_map_reset(gm_map* m, void* stream)
{
    clear_error();
    gm_status st = check_map(m);
    if (st != GM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    return map_clear(m, s);
}

gm_status gm_map_info(gm_map* m, int64_t* out)
{
    clear_error();
    gm_status st = check_map(m);
    if (st != GM_OK) return st;
    if (!out) return fail(GM_ERR_INVALID_ARGUMENT, "out is NULL");
    unsigned long long v[kMapCounters];
    GM_HIP(hipDeviceSynchronize());
    GM_HIP(hipMemcpy(v, m->counters.p, sizeof(v), hipMemcpyDeviceToHost));
    out[0] = (int64_t)v[2];
    out[1] = (int64_t)v[3];
    out[2] = (int64_t)v[4];
    out[3] = (int64_t)v[0];
    return GM_OK;
}

gm_status gm_map_destroy(gm_map* m)
{
    clear_error();
    if (!m) return GM_OK;
    const int dev = m->device;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != dev) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    delete m;
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
    return GM_OK;
}

}  // extern "C"
