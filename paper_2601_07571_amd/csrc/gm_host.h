// gm_host.h -- host-side state of the C ABI shared by capi.cpp and field_api.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "gazemap.h"
#include "gm_internal.h"

namespace gm {

gm_status fail(gm_status st, const char* fmt, ...);
void clear_error();
const char* last_error();

#define GM_HIP(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return gm::fail(GM_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Device buffer that only grows, or a borrowed range of memory owned elsewhere (never
// grown or freed: ensure() beyond its size fails).
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    hipError_t ensure(size_t want)
    {
        if (want <= bytes) return hipSuccess;
        if (borrowed) return hipErrorOutOfMemory;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        const size_t cap = want > 256 ? want : 256;
        hipError_t e = hipMalloc(&p, cap);
        if (e == hipSuccess) bytes = cap;
        return e;
    }
    void borrow(void* q, size_t n)
    {
        release();
        p = q;
        bytes = n;
        borrowed = true;
    }
    void release()
    {
        if (p && !borrowed) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        borrowed = false;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Pairs of HIP events around the kernels of one stage.
struct StageTimer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
    double total_ms = 0.0;
    int64_t launches = 0;
    hipError_t begin(hipStream_t s)
    {
        if (used == ev.size()) {
            hipEvent_t a, b;
            hipError_t e = hipEventCreate(&a);
            if (e != hipSuccess) return e;
            e = hipEventCreate(&b);
            if (e != hipSuccess) return e;
            ev.emplace_back(a, b);
        }
        return hipEventRecord(ev[used].first, s);
    }
    hipError_t end(hipStream_t s) { return hipEventRecord(ev[used++].second, s); }
    hipError_t collect()
    {
        for (size_t i = 0; i < used; ++i) {
            hipError_t e = hipEventSynchronize(ev[i].second);
            if (e != hipSuccess) return e;
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, ev[i].first, ev[i].second);
            if (e != hipSuccess) return e;
            total_ms += ms;
            ++launches;
        }
        used = 0;
        return hipSuccess;
    }
    void clear()
    {
        used = 0;
        total_ms = 0.0;
        launches = 0;
    }
    void release()
    {
        for (auto& p : ev) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
        ev.clear();
        clear();
    }
};

enum Stage { kStageSample = 0, kStagePrep, kStageDensity, kStageFinalize, kStages };
const char* const kStageNames[kStages] = {"sample", "prep", "density", "finalize"};

// Relative widening of kappa in the cheap cone gate.  The FP32 error of the gate value
// is below ~1e-6 |r|^2 (|e'| + |x'|)^2 (tile-local coordinates), the widening adds
// kGateWiden * kappa |p|^2 of margin, so no pair of the exact cone is missed while
// |p| > 0.46 R_tile; eyes closer than 2 R_tile to the tile origin take the exact
// path for every pair.  It enlarges the cone solid angle by about
// kGateWiden / (4 sigma)^2 (0.6 % at theta = 1 deg).
constexpr double kGateWiden = 3e-5;

// Device scratch of one density evaluation (one scene, one set of points and fixations).
struct DensityWork {
    // inv: the sorted position of every input point (input order)
    DevBuf fix, fx_shift, key, hist, cursor, scan_tmp, spos, smesh, inv, acc, max_acc, stats, zcam, zbuf;
    DevBuf bface, bcand;  // back-face rule data of the sorted points (see DensityLaunch::bface)
    bool backface = false;  // bface / bcand hold the current points' data
    int bits = 1;
    int64_t buckets = 8;
};

}  // namespace gm

using gm::DensityWork;
using gm::DevBuf;
using gm::BlasDesc;
using gm::HostBvh;
using gm::StageTimer;
using gm::kStages;

struct gm_scene {
    int device = 0;
    int32_t M = 0;
    int64_t T = 0, NV = 0;
    std::vector<int64_t> tri_off;  // [M+1]
    HostBvh bvh;
    // static device data
    DevBuf V, I, tri_mesh, tri_off_d, nodes, tris;
    // sampler state: FP64 areas, fixed-point weights W, their inclusive scan C, per-mesh
    // scale exponents S and weight totals do not depend on the sampling density, so they
    // are computed once per scene (weights_ready; totals and S also kept on the host,
    // where the per-density counts follow without a device round trip); counts and
    // offsets are rewritten by each sampling call; lat_* hold the lattice sampler's
    // per-triangle counts and their scan
    DevBuf area, W, C, max_bits, S, scan_tmp, counts, offsets, mesh_total, lat_W, lat_C;
    // the sampler's guide table (built with the weights): per mesh m, buckets of equal
    // width 2^gsh[m] in its target range, guide[goff[m] + k] = the triangle that the
    // bucket's lowest target selects, and one closing entry per mesh
    DevBuf guide, goff, gsh;
    bool weights_ready = false;
    std::vector<unsigned long long> mesh_total_h;
    std::vector<int32_t> S_h;
    // density scratch of the plain entry points
    DensityWork work;
    // meshes that bound a solid (gm_mesh_closed at creation; the caller may clear a
    // flag), on the host and the device, their bounding boxes (float4 lo, hi per mesh)
    // and the radius within which the back-face rule lists a point's neighbours
    std::vector<uint8_t> closed, closed_topology;
    DevBuf closed_d, mbox_d;
    float bf_rmax = 0.0f;
    bool any_closed() const
    {
        for (uint8_t c : closed)
            if (c) return true;
        return false;
    }
    // one BVH per mesh in the mesh's own frame (posed maps), built on first use:
    // BlasDesc per mesh into the concatenated node and record arrays (with copies)
    std::vector<BlasDesc> blas;
    DevBuf blas_nodes, blas_tris, blas_desc;
    // samples per lane of the plain density kernel; 0 = by occlusion mode (1 with a
    // visibility test, whose cost is per segment, 2 for the gate-only kernel)
    int32_t spl = 0;
    // fixations per work item of the plain density kernel; 0 = automatic (GM_FIX_PER_CHUNK)
    int32_t fix_per_chunk = 0;
    bool profiling = false;
    StageTimer timers[kStages];

    hipError_t tbegin(int st, hipStream_t s) { return profiling ? timers[st].begin(s) : hipSuccess; }
    hipError_t tend(int st, hipStream_t s)
    {
        if (!profiling) return hipSuccess;
        hipError_t e = timers[st].end(s);
        // keep the event list bounded when nobody reads it
        if (e == hipSuccess && timers[st].used >= 4096) e = timers[st].collect();
        return e;
    }

    ~gm_scene()
    {
        for (auto& t : timers) t.release();
        for (DevBuf* b : {&V, &I, &tri_mesh, &tri_off_d, &nodes, &tris, &area, &W, &C, &max_bits, &S, &scan_tmp,
                          &counts, &offsets, &mesh_total, &blas_nodes, &blas_tris, &blas_desc})
            b->release();
    }
};

namespace gm {
gm_status check_device(const gm_scene* sc);
// argument checks shared by accumulate_density and the batch planner
gm_status check_density_args(const gm_scene* sc, const float* pos, int64_t n, const gm_fixations* fix,
                             double theta_deg, uint32_t flags);
// allocate the scratch of one evaluation (not allowed while a stream is being captured)
gm_status density_reserve(DensityWork& w, int64_t n, int32_t F);
// queue fixation records, spatial sort and zeroed accumulators; fills `a` (chunking by
// fix_per_chunk, 0 = automatic) for launch_density / launch_density_queue
gm_status density_prep(gm_scene* sc, DensityWork& w, const float* pos, const int32_t* tri, const int32_t* mesh,
                       int64_t n, const gm_fixations* fix, double theta_deg, uint32_t mode, int spl,
                       int32_t fix_per_chunk, DensityLaunch& a, hipStream_t s);
// the back-face rule's data of the n sorted points from entry off of w (static scenes with
// a closed mesh and occlusion on; otherwise it marks the rule off)
gm_status density_backface(gm_scene* sc, DensityWork& w, int64_t n, uint32_t mode, hipStream_t s, int64_t off = 0);
// squared length of the longest segment the rule takes (see DensityLaunch::bf_L2max)
float backface_l2max(const gm_scene* sc);
// the two halves of density_prep's point side: zeroed accumulators and the spatial sort
// of the points into w (into entries [off, off + n), caller indices off + i); the
// launch descriptor for F records in w.fix
void density_sort(gm_scene* sc, DensityWork& w, const float* pos, const int32_t* tri, const int32_t* mesh,
                  int64_t n, hipStream_t s, int64_t off = 0);
void density_args(const gm_scene* sc, const DensityWork& w, int64_t n, int32_t F, double sigma, uint32_t mode,
                  int spl, int32_t fix_per_chunk, DensityLaunch& a);
// maximum and outputs
gm_status density_finalize(DensityWork& w, int64_t n, float* density, float* density_norm, float* max_out,
                           hipStream_t s);
// the scene's per-mesh BVHs (gm_scene::blas), built and uploaded once
gm_status ensure_blas(gm_scene* sc);
void zero(void* p, size_t bytes, hipStream_t s);
void fill_u32(void* p, int64_t n, uint32_t v, hipStream_t s);
}  // namespace gm
