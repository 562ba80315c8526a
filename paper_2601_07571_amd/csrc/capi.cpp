// capi.cpp -- the C ABI (include/gazemap.h): argument checks, scene upload,
// device scratch management and the launch sequence of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "gazemap.h"
#include "gm_host.h"
#include "gm_internal.h"

using namespace gm;

namespace gm {

namespace {
thread_local std::string g_error;
}  // namespace

gm_status fail(gm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

void clear_error() { g_error.clear(); }
const char* last_error() { return g_error.c_str(); }

}  // namespace gm

namespace gm {

gm_status check_device(const gm_scene* sc)
{
    int dev = -1;
    GM_HIP(hipGetDevice(&dev));
    if (dev != sc->device)
        return fail(GM_ERR_INVALID_ARGUMENT, "scene lives on device %d but device %d is current", sc->device, dev);
    return GM_OK;
}

namespace {
__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
}  // namespace

// fills by a kernel (also safe inside captured graphs)
void fill_u32(void* p, int64_t n, uint32_t v, hipStream_t s)
{
    if (n > 0) k_fill_u32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(static_cast<uint32_t*>(p), n, v);
}

void zero(void* p, size_t bytes, hipStream_t s) { fill_u32(p, (int64_t)((bytes + 3) / 4), 0u, s); }

}  // namespace gm

namespace {

// a1 + a2 on the device, once per scene: areas, weights, their scan and the per-mesh
// totals and scale exponents, the last two read back to the host (blocking, once).
gm_status ensure_weights(gm_scene* sc, hipStream_t s)
{
    if (sc->weights_ready) return GM_OK;
    const int64_t T = sc->T;
    const int32_t M = sc->M;
    GM_HIP(sc->area.ensure(sizeof(double) * T));
    GM_HIP(sc->W.ensure(8 * T));
    GM_HIP(sc->C.ensure(8 * T));
    GM_HIP(sc->max_bits.ensure(8 * M));
    GM_HIP(sc->S.ensure(4 * M));
    GM_HIP(sc->scan_tmp.ensure(scan_tmp_bytes(T)));
    GM_HIP(sc->counts.ensure(8 * M));
    GM_HIP(sc->offsets.ensure(8 * (M + 1)));
    GM_HIP(sc->mesh_total.ensure(8 * M));
    GM_HIP(sc->tbegin(kStageSample, s));
    zero(sc->max_bits.p, 8 * (size_t)M, s);
    launch_tri_area(sc->V.as<float>(), sc->I.as<int32_t>(), sc->tri_mesh.as<int32_t>(), T, sc->area.as<double>(),
                    sc->max_bits.as<unsigned long long>(), s);
    launch_mesh_scale(sc->max_bits.as<unsigned long long>(), sc->tri_off_d.as<int64_t>(), M, sc->S.as<int32_t>(), s);
    launch_tri_weight(sc->area.as<double>(), sc->tri_mesh.as<int32_t>(), sc->S.as<int32_t>(), T,
                      sc->W.as<unsigned long long>(), s);
    launch_inclusive_scan_u64(sc->W.as<unsigned long long>(), sc->C.as<unsigned long long>(), T, sc->scan_tmp.p, s);
    // the totals (the counts of density 0 are unused)
    launch_mesh_counts(sc->C.as<unsigned long long>(), sc->tri_off_d.as<int64_t>(), sc->S.as<int32_t>(), M, 0.0,
                       sc->counts.as<int64_t>(), sc->offsets.as<int64_t>(), sc->mesh_total.as<unsigned long long>(), s);
    GM_HIP(hipGetLastError());
    GM_HIP(sc->tend(kStageSample, s));
    sc->mesh_total_h.assign((size_t)M, 0ull);
    sc->S_h.assign((size_t)M, 0);
    GM_HIP(hipMemcpyAsync(sc->mesh_total_h.data(), sc->mesh_total.p, 8 * (size_t)M, hipMemcpyDeviceToHost, s));
    GM_HIP(hipMemcpyAsync(sc->S_h.data(), sc->S.p, 4 * (size_t)M, hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    // the guide table: per mesh about one bucket per triangle (a power of two >= its
    // triangle count, at most 2^24), each 2^gsh targets wide, plus a closing entry
    std::vector<int64_t> goff((size_t)M + 1, 0);
    std::vector<int32_t> gsh((size_t)M, 0);
    for (int32_t m = 0; m < M; ++m) {
        const int64_t nt = sc->tri_off[(size_t)m + 1] - sc->tri_off[(size_t)m];
        int g = 0;
        while (g < 24 && ((int64_t)1 << g) < nt) ++g;
        const unsigned long long tot = sc->mesh_total_h[(size_t)m];
        int len = 0;  // bit length of tot - 1: targets lie in [0, tot)
        for (unsigned long long v = tot > 1 ? tot - 1 : 0; v; v >>= 1) ++len;
        gsh[(size_t)m] = std::max(0, len - g);
        const int64_t buckets = tot > 0 ? (int64_t)((tot - 1) >> gsh[(size_t)m]) + 1 : 1;
        goff[(size_t)m + 1] = goff[(size_t)m] + buckets + 1;
    }
    GM_HIP(sc->goff.ensure(8 * ((size_t)M + 1)));
    GM_HIP(sc->gsh.ensure(4 * (size_t)M));
    GM_HIP(sc->guide.ensure(4 * (size_t)goff[(size_t)M]));
    GM_HIP(hipMemcpyAsync(sc->goff.p, goff.data(), 8 * ((size_t)M + 1), hipMemcpyHostToDevice, s));
    GM_HIP(hipMemcpyAsync(sc->gsh.p, gsh.data(), 4 * (size_t)M, hipMemcpyHostToDevice, s));
    launch_sample_guide(sc->C.as<unsigned long long>(), sc->tri_off_d.as<int64_t>(), sc->goff.as<int64_t>(),
                        sc->gsh.as<int32_t>(), M, goff[(size_t)M], sc->guide.as<int32_t>(), s);
    GM_HIP(hipGetLastError());
    GM_HIP(hipStreamSynchronize(s));  // the host vectors above go out of scope
    sc->weights_ready = true;
    return GM_OK;
}

// Per-mesh counts round(k * W_m 2^-S_m), evaluated on the host exactly as k_mesh_counts
// evaluates them on the device (the same FP64 operations in the same order).
gm_status sample_counts(gm_scene* sc, double k, hipStream_t s, std::vector<int64_t>& counts)
{
    if (!(k > 0.0) || !std::isfinite(k)) return fail(GM_ERR_INVALID_ARGUMENT, "samples_per_m2 must be finite and > 0");
    gm_status st = ensure_weights(sc, s);
    if (st != GM_OK) return st;
    counts.assign((size_t)sc->M, 0);
    for (int32_t m = 0; m < sc->M; ++m) {
        const unsigned long long tot = sc->mesh_total_h[(size_t)m];
        const double area = std::ldexp((double)tot, -sc->S_h[(size_t)m]);
        counts[(size_t)m] = tot ? (int64_t)std::floor(area * k + 0.5) : 0;
    }
    return GM_OK;
}

// Lattice sampler counts: areas (a1, cached), Eq. (4) resolutions and Eq. (1) counts
// per triangle, their inclusive scan in sc->lat_C, per-mesh totals (blocking).
gm_status lattice_counts(gm_scene* sc, double k, hipStream_t s, std::vector<int64_t>& counts)
{
    if (!(k > 0.0) || !(k <= 1e12)) return fail(GM_ERR_INVALID_ARGUMENT, "samples_per_m2 must be in (0, 1e12]");
    gm_status st = ensure_weights(sc, s);
    if (st != GM_OK) return st;
    const int64_t T = sc->T;
    const int32_t M = sc->M;
    GM_HIP(sc->lat_W.ensure(8 * T));
    GM_HIP(sc->lat_C.ensure(8 * T));
    GM_HIP(sc->tbegin(kStageSample, s));
    launch_lattice_count(sc->area.as<double>(), T, k, sc->lat_W.as<unsigned long long>(), s);
    launch_inclusive_scan_u64(sc->lat_W.as<unsigned long long>(), sc->lat_C.as<unsigned long long>(), T,
                              sc->scan_tmp.p, s);
    launch_lattice_mesh_counts(sc->lat_C.as<unsigned long long>(), sc->tri_off_d.as<int64_t>(), M,
                               sc->counts.as<int64_t>(), s);
    GM_HIP(hipGetLastError());
    GM_HIP(sc->tend(kStageSample, s));
    counts.assign((size_t)M, 0);
    GM_HIP(hipMemcpyAsync(counts.data(), sc->counts.p, 8 * (size_t)M, hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    return GM_OK;
}

bool finite3(const float* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

}  // namespace

namespace gm {

gm_status check_density_args(const gm_scene* sc, const float* pos, int64_t n, const gm_fixations* fix,
                             double theta_deg, uint32_t flags)
{
    if (!sc) return fail(GM_ERR_INVALID_ARGUMENT, "scene is NULL");
    if (!fix) return fail(GM_ERR_INVALID_ARGUMENT, "fixations is NULL");
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GM_ERR_INVALID_ARGUMENT, "n must be in [0, 2^31)");
    if (n > 0 && !pos) return fail(GM_ERR_INVALID_ARGUMENT, "pos is NULL");
    if (fix->n < 0) return fail(GM_ERR_INVALID_ARGUMENT, "fixation count < 0");
    if (fix->n > 0 && (!fix->eye || !fix->gaze || !fix->duration))
        return fail(GM_ERR_INVALID_ARGUMENT, "fixation arrays must not be NULL");
    if (!(theta_deg > 0.0 && theta_deg < 45.0)) return fail(GM_ERR_INVALID_ARGUMENT, "theta_deg must be in (0, 45)");
    const uint32_t mode = flags & GM_OCC_MASK;
    if (mode > GM_OCC_FULL || (flags & ~GM_OCC_MASK)) return fail(GM_ERR_INVALID_ARGUMENT, "unknown flags 0x%x", flags);
    return check_device(sc);
}

gm_status density_reserve(DensityWork& w, int64_t n, int32_t F)
{
    // spatial buckets: about one sample per bucket of the scene's box, at most 2^21; launches
    // of more than 2^20 points take 2^24, of more than 2^23 points 2^27.  Samples lie on
    // surfaces, so an occupied bucket of the coarser grid holds about a hundred of them in no
    // particular order (the scatter's atomic cursor) and a wave's 64 segments would start
    // anywhere in it: the finer grids cut node visits by 6 % on the paper-shaped map (2M
    // points) and by 10 % on the scale-up map (20M points).
    int bits = 1;
    while (bits < 7 && ((int64_t)1 << (3 * bits)) < n) ++bits;
    if (n > ((int64_t)1 << 20)) bits = 8;
    if (n > ((int64_t)1 << 23)) bits = 9;
    w.bits = bits;
    w.buckets = (int64_t)1 << (3 * bits);
    const int64_t nn = std::max<int64_t>(n, 1);
    GM_HIP(w.fix.ensure(sizeof(FixRec) * (size_t)std::max(F, 1)));
    GM_HIP(w.fx_shift.ensure(16));
    GM_HIP(w.key.ensure(4 * nn));
    GM_HIP(w.hist.ensure(4 * w.buckets));
    GM_HIP(w.cursor.ensure(4 * w.buckets));
    GM_HIP(w.scan_tmp.ensure(scan_tmp_bytes(w.buckets)));
    GM_HIP(w.spos.ensure(16 * nn));
    GM_HIP(w.smesh.ensure(4 * nn));
    GM_HIP(w.inv.ensure(4 * nn));
    GM_HIP(w.acc.ensure(8 * nn));
    GM_HIP(w.max_acc.ensure(8));
    GM_HIP(w.stats.ensure(8 * kDensityStats));
    return GM_OK;
}

void density_sort(gm_scene* sc, DensityWork& w, const float* pos, const int32_t* tri, const int32_t* mesh,
                  int64_t n, hipStream_t s, int64_t off)
{
    if (n <= 0) return;
    zero(w.acc.as<unsigned long long>() + off, 8 * (size_t)n, s);
    zero(w.hist.p, 4 * (size_t)w.buckets, s);
    float lo[3];
    float ext = 0.0f;
    for (int c = 0; c < 3; ++c) {
        lo[c] = sc->bvh.lo[c];
        ext = std::max(ext, sc->bvh.hi[c] - sc->bvh.lo[c]);
    }
    const int cells = 1 << w.bits;
    const float inv_cell = ext > 0.0f ? (float)cells / ext : 1.0f;
    launch_morton(pos, tri, mesh, sc->tri_mesh.as<int32_t>(), n, lo, inv_cell, w.bits, w.key.as<uint32_t>(),
                  w.hist.as<uint32_t>(), s);
    launch_exclusive_scan_u32(w.hist.as<uint32_t>(), w.cursor.as<uint32_t>(), w.buckets, w.scan_tmp.p, s);
    launch_scatter(pos, tri, mesh, sc->tri_mesh.as<int32_t>(), sc->T, n, w.key.as<uint32_t>(),
                   w.cursor.as<uint32_t>(), w.spos.as<float4>() + off, w.smesh.as<int32_t>() + off,
                   w.inv.as<int32_t>() + off, (int32_t)off, s);
}

void density_args(const gm_scene* sc, const DensityWork& w, int64_t n, int32_t F, double sigma, uint32_t mode,
                  int spl, int32_t fix_per_chunk, DensityLaunch& a)
{
    a.spos = w.spos.as<float4>();
    a.smesh = w.smesh.as<int32_t>();
    a.n = n;
    a.fix = w.fix.as<FixRec>();
    a.F = F;
    a.nodes = sc->nodes.as<BvhNode>();
    a.node_stride = (int64_t)sc->bvh.nodes.size();
    a.tris = sc->tris.as<BvhTri>();
    a.tri_stride = (int64_t)sc->bvh.tris.size();
    a.occ_mode = (int32_t)mode;
    a.cone2 = (float)(16.0 * sigma * sigma);
    a.kexp = (float)(1.0 / (2.0 * sigma * sigma * std::log(2.0)));
    a.fx_shift = w.fx_shift.as<int32_t>();
    a.acc = w.acc.as<unsigned long long>();
    a.stats = w.stats.as<unsigned long long>();
    a.spl = spl;
    if (fix_per_chunk <= 0) {
        // The cost of a (tile, chunk) item varies a lot (how many of its fixations see
        // the tile), so the grid holds many small items: at least ~512k of them and at
        // most 1024 fixations each, but chunks of no fewer than 128 fixations.  Without
        // a visibility test an item costs little beyond its fixed part (its samples,
        // the staging and the tile cone test of every fixation, the flush), so chunks
        // are at least 512 fixations long there (the paper-shaped gate: 2.43 ms at 128,
        // 1.71 ms at 512, 1.74 ms at 1024).
        const int64_t tiles = std::max<int64_t>(1, (n + 256 * spl - 1) / (256 * spl));
        const int64_t min_chunk = mode == GM_OCC_NONE ? 512 : 128;
        const int64_t max_chunks = std::max<int64_t>(1, (F + min_chunk - 1) / min_chunk);
        const int64_t want = std::max<int64_t>((524288 + tiles - 1) / tiles, (F + 1023) / 1024);
        // the grid is tiles x chunks: chunks <= 65535 (grid y) and tiles x chunks < 2^31
        const int64_t cap = std::min<int64_t>(65535, std::max<int64_t>(1, INT32_MAX / tiles));
        const int64_t chunks = std::min<int64_t>(std::min(max_chunks, cap), std::max<int64_t>(1, want));
        fix_per_chunk = (int32_t)std::max<int64_t>(1, (F + chunks - 1) / chunks);
    }
    a.fix_per_chunk = fix_per_chunk;
    a.n_chunks = F > 0 ? (int32_t)((F + fix_per_chunk - 1) / fix_per_chunk) : 0;
    a.F_live = nullptr;
    if (w.backface && mode != GM_OCC_NONE) {
        a.bface = w.bface.as<float4>();
        a.bcand = w.bcand.as<int32_t>();
        a.mbox = sc->mbox_d.as<float4>();
        a.bf_tris = sc->tris.as<BvhTri>() + 2 * sc->bvh.tris.size();
        a.bf_L2max = backface_l2max(sc);
    }
}

float backface_l2max(const gm_scene* sc)
{
    // the rule's longest segment: its last kEpsV stretch stays 1e-3 inside rmax
    const double lmax = (double)sc->bf_rmax / kEpsV * (1.0 - 1e-3);
    return (float)(lmax * lmax);
}

gm_status density_backface(gm_scene* sc, DensityWork& w, int64_t n, uint32_t mode, hipStream_t s, int64_t off)
{
    w.backface = false;
    if (mode == GM_OCC_NONE || !sc->any_closed() || n <= 0) return GM_OK;
    GM_HIP(w.bface.ensure(16 * (size_t)(off + n)));
    GM_HIP(w.bcand.ensure(4 * (size_t)kBfCand * (size_t)(off + n)));
    launch_backface_prep(w.spos.as<float4>() + off, w.smesh.as<int32_t>() + off, n, sc->V.as<float>(),
                         sc->I.as<int32_t>(), sc->closed_d.as<uint8_t>(), sc->nodes.as<BvhNode>(),
                         sc->tris.as<BvhTri>() + 2 * sc->bvh.tris.size(), sc->bf_rmax, w.bface.as<float4>() + off,
                         w.bcand.as<int32_t>() + kBfCand * off, s);
    GM_HIP(hipGetLastError());
    w.backface = true;
    return GM_OK;
}

gm_status density_prep(gm_scene* sc, DensityWork& w, const float* pos, const int32_t* tri, const int32_t* mesh,
                       int64_t n, const gm_fixations* fix, double theta_deg, uint32_t mode, int spl,
                       int32_t fix_per_chunk, DensityLaunch& a, hipStream_t s)
{
    const int32_t F = fix->n;
    const double sigma = std::tan(theta_deg * M_PI / 180.0);
    zero(w.stats.p, 8 * kDensityStats, s);
    zero(w.fx_shift.p, 16, s);
    zero(w.max_acc.p, 8, s);
    launch_fix_prep(fix->eye, fix->gaze, fix->duration, F, sigma, kGateWiden, w.fix.as<FixRec>(), nullptr,
                    w.fx_shift.as<int32_t>(), s);
    density_sort(sc, w, pos, tri, mesh, n, s);
    gm_status st = density_backface(sc, w, n, mode, s);
    if (st != GM_OK) return st;
    density_args(sc, w, n, F, sigma, mode, spl, fix_per_chunk, a);
    GM_HIP(hipGetLastError());
    return GM_OK;
}

gm_status density_finalize(DensityWork& w, int64_t n, float* density, float* density_norm, float* max_out,
                           hipStream_t s)
{
    launch_finalize(w.acc.as<unsigned long long>(), w.inv.as<int32_t>(), n, w.fx_shift.as<int32_t>(),
                    w.max_acc.as<unsigned long long>(), density, density_norm, max_out, s);
    GM_HIP(hipGetLastError());
    return GM_OK;
}

}  // namespace gm

extern "C" {

const char* gm_last_error(void) { return gm::last_error(); }

int32_t gm_version(void) { return (1 << 16) | 0; }

gm_status gm_scene_create(const gm_mesh* meshes, int32_t n_meshes, gm_scene** out)
{
    gm::clear_error();
    if (!out) return fail(GM_ERR_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    if (!meshes || n_meshes < 1 || n_meshes > 4096)
        return fail(GM_ERR_INVALID_ARGUMENT, "n_meshes must be in [1, 4096] (got %d)", n_meshes);
    int64_t T = 0, NV = 0;
    for (int32_t m = 0; m < n_meshes; ++m) {
        const gm_mesh& g = meshes[m];
        if (!g.vertices || !g.indices || g.n_vertices < 3 || g.n_triangles < 1)
            return fail(GM_ERR_INVALID_ARGUMENT, "mesh %d: needs >= 3 vertices and >= 1 triangle", m);
        for (int64_t v = 0; v < g.n_vertices; ++v)
            if (!finite3(g.vertices + 3 * v)) return fail(GM_ERR_INVALID_ARGUMENT, "mesh %d: vertex %lld not finite", m, (long long)v);
        for (int64_t t = 0; t < 3 * (int64_t)g.n_triangles; ++t)
            if (g.indices[t] < 0 || g.indices[t] >= g.n_vertices)
                return fail(GM_ERR_INVALID_ARGUMENT, "mesh %d: index %d out of range", m, g.indices[t]);
        T += g.n_triangles;
        NV += g.n_vertices;
    }
    if (T >= (int64_t)1 << 31) return fail(GM_ERR_INVALID_ARGUMENT, "more than 2^31 - 1 triangles");
    gm_scene* sc = new (std::nothrow) gm_scene();
    if (!sc) return fail(GM_ERR_OUT_OF_MEMORY, "host allocation failed");
    if (const char* e = std::getenv("GM_FIX_PER_CHUNK")) sc->fix_per_chunk = std::max(0, std::atoi(e));
    if (const char* e = std::getenv("GM_SAMPLES_PER_LANE")) {
        const int v = std::atoi(e);
        if (v == 1 || v == 2 || v == 4) sc->spl = v;
    }
    hipError_t he = hipGetDevice(&sc->device);
    if (he != hipSuccess) {
        delete sc;
        return fail(GM_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(he));
    }
    sc->M = n_meshes;
    sc->T = T;
    sc->NV = NV;
    std::vector<float> V((size_t)NV * 3);
    std::vector<int32_t> I((size_t)T * 3), tm((size_t)T);
    sc->tri_off.assign((size_t)n_meshes + 1, 0);
    int64_t vb = 0, tb = 0;
    for (int32_t m = 0; m < n_meshes; ++m) {
        const gm_mesh& g = meshes[m];
        std::memcpy(V.data() + 3 * vb, g.vertices, sizeof(float) * 3 * (size_t)g.n_vertices);
        for (int64_t t = 0; t < g.n_triangles; ++t) {
            for (int k = 0; k < 3; ++k) I[(size_t)(3 * (tb + t) + k)] = (int32_t)(g.indices[3 * t + k] + vb);
            tm[(size_t)(tb + t)] = m;
        }
        sc->tri_off[(size_t)m] = tb;
        vb += g.n_vertices;
        tb += g.n_triangles;
    }
    sc->tri_off[(size_t)n_meshes] = tb;
    int leaf_max = kLeafMax;
    if (const char* e = std::getenv("GM_BVH_LEAF")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= kLeafMax) leaf_max = v;
    }
    build_bvh(V.data(), I.data(), tm.data(), T, sc->bvh, leaf_max);
    // meshes that bound a solid, their boxes, and the back-face rule's neighbour radius:
    // kEpsV of twice the scene's diagonal plus 4 m (segments up to that length, eyes within
    // a few metres of the scene, use the rule)
    sc->closed.assign((size_t)n_meshes, 0);
    std::vector<float> mbox((size_t)8 * n_meshes, 0.0f);
    for (int32_t m = 0; m < n_meshes; ++m) {
        const gm_mesh& g = meshes[m];
        sc->closed[(size_t)m] = mesh_is_closed(g.vertices, g.n_vertices, g.indices, g.n_triangles) ? 1 : 0;
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t t = 0; t < 3 * (int64_t)g.n_triangles; ++t)
            for (int c = 0; c < 3; ++c) {
                const float v = g.vertices[3 * (int64_t)g.indices[t] + c];
                lo[c] = std::min(lo[c], v);
                hi[c] = std::max(hi[c], v);
            }
        for (int c = 0; c < 3; ++c) {
            mbox[(size_t)8 * m + c] = lo[c];
            mbox[(size_t)8 * m + 4 + c] = hi[c];
        }
    }
    sc->closed_topology = sc->closed;
    {
        double d2 = 0.0;
        for (int c = 0; c < 3; ++c) d2 += ((double)sc->bvh.hi[c] - sc->bvh.lo[c]) * ((double)sc->bvh.hi[c] - sc->bvh.lo[c]);
        sc->bf_rmax = (float)(kEpsV * (2.0 * std::sqrt(d2) + 4.0));
    }

    auto up = [&](DevBuf& b, const void* src, size_t bytes) -> hipError_t {
        hipError_t e = b.ensure(bytes);
        if (e != hipSuccess) return e;
        return hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(sc->V, V.data(), V.size() * 4);
    if (e == hipSuccess) e = up(sc->I, I.data(), I.size() * 4);
    if (e == hipSuccess) e = up(sc->tri_mesh, tm.data(), tm.size() * 4);
    if (e == hipSuccess) e = up(sc->tri_off_d, sc->tri_off.data(), sc->tri_off.size() * 8);
    std::vector<BvhNode> node8;
    octant_node_copies(sc->bvh.nodes, node8);
    if (e == hipSuccess) e = up(sc->nodes, node8.data(), node8.size() * sizeof(BvhNode));
    std::vector<BvhTri> tri3;
    permute_tri_copies(sc->bvh.tris, tri3);
    if (e == hipSuccess) e = up(sc->tris, tri3.data(), tri3.size() * sizeof(BvhTri));
    if (e == hipSuccess) e = up(sc->closed_d, sc->closed.data(), sc->closed.size());
    if (e == hipSuccess) e = up(sc->mbox_d, mbox.data(), mbox.size() * 4);
    if (e != hipSuccess) {
        delete sc;
        return fail(e == hipErrorOutOfMemory ? GM_ERR_OUT_OF_MEMORY : GM_ERR_DEVICE, "scene upload: %s",
                    hipGetErrorString(e));
    }
    *out = sc;
    return GM_OK;
}

gm_status gm_scene_destroy(gm_scene* scene)
{
    gm::clear_error();
    if (scene) {
        (void)hipDeviceSynchronize();
        delete scene;
    }
    return GM_OK;
}

gm_status gm_scene_info(const gm_scene* sc, int64_t* n_triangles, int32_t* n_meshes, int64_t* n_bvh_nodes,
                        int32_t* bvh_depth, float* bbox)
{
    gm::clear_error();
    if (!sc) return fail(GM_ERR_INVALID_ARGUMENT, "scene is NULL");
    if (n_triangles) *n_triangles = sc->T;
    if (n_meshes) *n_meshes = sc->M;
    if (n_bvh_nodes) *n_bvh_nodes = (int64_t)sc->bvh.nodes.size();
    if (bvh_depth) *bvh_depth = sc->bvh.depth;
    if (bbox)
        for (int a = 0; a < 3; ++a) {
            bbox[a] = sc->bvh.lo[a];
            bbox[3 + a] = sc->bvh.hi[a];
        }
    return GM_OK;
}

gm_status gm_scene_mesh_closed(const gm_scene* sc, uint8_t* closed)
{
    gm::clear_error();
    if (!sc || !closed) return fail(GM_ERR_INVALID_ARGUMENT, "scene and closed must not be NULL");
    std::memcpy(closed, sc->closed.data(), sc->closed.size());
    return GM_OK;
}

gm_status gm_scene_set_mesh_closed(gm_scene* sc, int32_t mesh, int32_t closed)
{
    gm::clear_error();
    if (!sc) return fail(GM_ERR_INVALID_ARGUMENT, "scene is NULL");
    if (mesh < 0 || mesh >= sc->M) return fail(GM_ERR_INVALID_ARGUMENT, "mesh %d outside [0, %d)", mesh, sc->M);
    if (closed && !sc->closed_topology[(size_t)mesh])
        return fail(GM_ERR_INVALID_ARGUMENT, "mesh %d does not bound a solid (gm_mesh_closed)", mesh);
    gm_status st = check_device(sc);
    if (st != GM_OK) return st;
    GM_HIP(hipDeviceSynchronize());
    sc->closed[(size_t)mesh] = closed ? 1 : 0;
    GM_HIP(hipMemcpy(sc->closed_d.as<uint8_t>() + mesh, &sc->closed[(size_t)mesh], 1, hipMemcpyHostToDevice));
    return GM_OK;
}

gm_status gm_count_lattice_samples(gm_scene* sc, double k, int64_t* n_per_mesh, void* stream)
{
    gm::clear_error();
    if (!sc || !n_per_mesh) return fail(GM_ERR_INVALID_ARGUMENT, "scene and n_per_mesh must not be NULL");
    gm_status st = check_device(sc);
    if (st != GM_OK) return st;
    std::vector<int64_t> counts;
    st = lattice_counts(sc, k, (hipStream_t)stream, counts);
    if (st != GM_OK) return st;
    std::memcpy(n_per_mesh, counts.data(), 8 * counts.size());
    return GM_OK;
}

gm_status build_lattice_samples(gm_scene* sc, double k, int32_t* tri, int32_t* mesh, float* bary, float* pos,
                                int64_t capacity, int64_t* n_out, void* stream)
{
    gm::clear_error();
    if (!sc) return fail(GM_ERR_INVALID_ARGUMENT, "scene is NULL");
    if (capacity < 0) return fail(GM_ERR_INVALID_ARGUMENT, "capacity < 0");
    gm_status st = check_device(sc);
    if (st != GM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> counts;
    st = lattice_counts(sc, k, s, counts);
    if (st != GM_OK) return st;
    int64_t N = 0;
    for (int64_t c : counts) N += c;
    if (n_out) *n_out = N;
    if (N > capacity) return fail(GM_ERR_CAPACITY, "%lld samples do not fit capacity %lld", (long long)N, (long long)capacity);
    if (N >= (int64_t)1 << 31) return fail(GM_ERR_INVALID_ARGUMENT, "more than 2^31 - 1 samples");
    GM_HIP(sc->tbegin(kStageSample, s));
    launch_lattice_sample(sc->V.as<float>(), sc->I.as<int32_t>(), sc->tri_mesh.as<int32_t>(), sc->area.as<double>(),
                          sc->lat_C.as<unsigned long long>(), sc->T, N, k, tri, mesh, bary, pos, s);
    GM_HIP(hipGetLastError());
    GM_HIP(sc->tend(kStageSample, s));
    return GM_OK;
}

gm_status gm_count_surface_samples(gm_scene* sc, double k, int64_t* n_per_mesh, void* stream)
{
    gm::clear_error();
    if (!sc || !n_per_mesh) return fail(GM_ERR_INVALID_ARGUMENT, "scene and n_per_mesh must not be NULL");
    gm_status st = check_device(sc);
    if (st != GM_OK) return st;
    std::vector<int64_t> counts;
    st = sample_counts(sc, k, (hipStream_t)stream, counts);
    if (st != GM_OK) return st;
    std::memcpy(n_per_mesh, counts.data(), 8 * counts.size());
    return GM_OK;
}

gm_status build_surface_samples(gm_scene* sc, double k, uint64_t seed, int32_t* tri, int32_t* mesh, float* bary,
                                float* pos, int64_t capacity, int64_t* n_out, void* stream)
{
    gm::clear_error();
    if (!sc) return fail(GM_ERR_INVALID_ARGUMENT, "scene is NULL");
    if (capacity < 0) return fail(GM_ERR_INVALID_ARGUMENT, "capacity < 0");
    gm_status st = check_device(sc);
    if (st != GM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> counts;
    st = sample_counts(sc, k, s, counts);
    if (st != GM_OK) return st;
    int64_t N = 0;
    for (int64_t c : counts) N += c;
    if (n_out) *n_out = N;
    if (N > capacity) return fail(GM_ERR_CAPACITY, "%lld samples do not fit capacity %lld", (long long)N, (long long)capacity);
    if (N >= (int64_t)1 << 31) return fail(GM_ERR_INVALID_ARGUMENT, "more than 2^31 - 1 samples");
    GM_HIP(sc->tbegin(kStageSample, s));
    launch_mesh_counts(sc->C.as<unsigned long long>(), sc->tri_off_d.as<int64_t>(), sc->S.as<int32_t>(), sc->M, k,
                       sc->counts.as<int64_t>(), sc->offsets.as<int64_t>(), sc->mesh_total.as<unsigned long long>(), s);
    launch_sample(sc->V.as<float>(), sc->I.as<int32_t>(), sc->C.as<unsigned long long>(), sc->tri_off_d.as<int64_t>(),
                  sc->offsets.as<int64_t>(), sc->mesh_total.as<unsigned long long>(), sc->guide.as<int32_t>(),
                  sc->goff.as<int64_t>(), sc->gsh.as<int32_t>(), sc->M, N, seed, tri, mesh, bary, pos, s);
    GM_HIP(hipGetLastError());
    GM_HIP(sc->tend(kStageSample, s));
    return GM_OK;
}

gm_status accumulate_density(gm_scene* sc, const float* pos, const int32_t* tri, const int32_t* mesh, int64_t n,
                             const gm_fixations* fix, double theta_deg, uint32_t flags, float* density,
                             float* density_norm, float* max_out, void* stream)
{
    gm::clear_error();
    gm_status st = check_density_args(sc, pos, n, fix, theta_deg, flags);
    if (st != GM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    DensityWork& w = sc->work;
    st = density_reserve(w, n, fix->n);
    if (st != GM_OK) return st;
    DensityLaunch a;
    GM_HIP(sc->tbegin(kStagePrep, s));
    const int spl = sc->spl ? sc->spl : ((flags & GM_OCC_MASK) != GM_OCC_NONE ? 1 : 2);
    st = density_prep(sc, w, pos, tri, mesh, n, fix, theta_deg, flags & GM_OCC_MASK, spl, sc->fix_per_chunk, a, s);
    if (st != GM_OK) return st;

    GM_HIP(sc->tend(kStagePrep, s));
    if (n > 0 && fix->n > 0) {
        GM_HIP(sc->tbegin(kStageDensity, s));
        launch_density(a, s);
        GM_HIP(sc->tend(kStageDensity, s));
    }
    GM_HIP(sc->tbegin(kStageFinalize, s));
    st = density_finalize(w, n, density, density_norm, max_out, s);
    if (st != GM_OK) return st;
    GM_HIP(sc->tend(kStageFinalize, s));
    return GM_OK;
}

gm_status gm_debug_sqrt_f64(const double* x, double* y, int64_t n, void* stream)
{
    gm::clear_error();
    if (n < 0 || (n > 0 && (!x || !y))) return fail(GM_ERR_INVALID_ARGUMENT, "NULL argument or negative size");
    launch_sqrt_f64(x, y, n, (hipStream_t)stream);
    GM_HIP(hipGetLastError());
    return GM_OK;
}

gm_status gm_debug_pair_values(const float* pos, int64_t n_points, const gm_fixations* fix, double theta_deg,
                               const int32_t* pair_s, const int32_t* pair_f, int64_t m, float* g_out, void* stream)
{
    gm::clear_error();
    if (!fix || (m > 0 && (!pos || !pair_s || !pair_f || !g_out)) || m < 0 || n_points < 0 || fix->n < 0)
        return fail(GM_ERR_INVALID_ARGUMENT, "NULL argument or negative size");
    if (!(theta_deg > 0.0 && theta_deg < 45.0)) return fail(GM_ERR_INVALID_ARGUMENT, "theta_deg must be in (0, 45)");
    hipStream_t s = (hipStream_t)stream;
    const double sigma = std::tan(theta_deg * M_PI / 180.0);
    DevBuf rec, sh;
    GM_HIP(rec.ensure(sizeof(FixRec) * (size_t)std::max(fix->n, 1)));
    GM_HIP(sh.ensure(16));
    zero(sh.p, 16, s);
    launch_fix_prep(fix->eye, fix->gaze, fix->duration, fix->n, sigma, kGateWiden, rec.as<FixRec>(), nullptr,
                    sh.as<int32_t>(), s);
    launch_pair_values(pos, rec.as<FixRec>(), pair_s, pair_f, m, n_points, fix->n, (float)(16.0 * sigma * sigma),
                       (float)(1.0 / (2.0 * sigma * sigma * std::log(2.0))), g_out, s);
    hipError_t e = hipStreamSynchronize(s);
    rec.release();
    sh.release();
    GM_HIP(e);
    GM_HIP(hipGetLastError());
    return GM_OK;
}

gm_status gm_debug_pair_visibility(gm_scene* sc, const float* pos, const int32_t* tri, const int32_t* mesh,
                                   int64_t n_points, const float* eye, const float* gaze, int32_t n_eyes,
                                   const int32_t* pair_s, const int32_t* pair_f, int64_t m, uint32_t flags,
                                   uint8_t* vis_out, void* stream)
{
    gm::clear_error();
    if (!sc || m < 0 || n_points < 0 || n_eyes < 0 || (m > 0 && (!pos || !eye || !pair_s || !pair_f || !vis_out)))
        return fail(GM_ERR_INVALID_ARGUMENT, "NULL argument or negative size");
    const uint32_t mode = flags & GM_OCC_MASK;
    if (mode > GM_OCC_FULL) return fail(GM_ERR_INVALID_ARGUMENT, "unknown occlusion mode");
    gm_status st = check_device(sc);
    if (st != GM_OK) return st;
    BackfaceArgs bf;
    if (sc->any_closed()) {
        bf.V = sc->V.as<float>();
        bf.I = sc->I.as<int32_t>();
        bf.closed = sc->closed_d.as<uint8_t>();
        bf.mbox = sc->mbox_d.as<float4>();
        bf.rmax = sc->bf_rmax;
        bf.l2max = backface_l2max(sc);
    }
    launch_pair_visibility(pos, tri, mesh, sc->tri_mesh.as<int32_t>(), eye, gaze, pair_s, pair_f, m, n_points, n_eyes,
                           sc->T, sc->nodes.as<BvhNode>(), sc->tris.as<BvhTri>() + 2 * sc->bvh.tris.size(),
                           (int32_t)mode, bf, vis_out, (hipStream_t)stream);
    GM_HIP(hipGetLastError());
    return GM_OK;
}

gm_status gm_density_counters(gm_scene* sc, int64_t* out, int32_t n_out)
{
    gm::clear_error();
    if (!sc || !out) return fail(GM_ERR_INVALID_ARGUMENT, "scene and out must not be NULL");
    if (n_out < 0) return fail(GM_ERR_INVALID_ARGUMENT, "n_out < 0");
    const int n = std::min<int32_t>(n_out, kDensityStats);
    for (int i = 0; i < n_out; ++i) out[i] = 0;
    if (!sc->work.stats.p) return GM_OK;
    GM_HIP(hipDeviceSynchronize());
    unsigned long long v[kDensityStats];
    GM_HIP(hipMemcpy(v, sc->work.stats.p, sizeof(v), hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) out[i] = (int64_t)v[i];
    return GM_OK;
}

gm_status gm_density_stats(gm_scene* sc, int64_t* out) { return gm_density_counters(sc, out, 4); }

gm_status gm_profile_enable(gm_scene* sc, int32_t on)
{
    gm::clear_error();
    if (!sc) return fail(GM_ERR_INVALID_ARGUMENT, "scene is NULL");
    for (auto& t : sc->timers) {
        GM_HIP(t.collect());
        t.clear();
    }
    sc->profiling = on != 0;
    return GM_OK;
}

gm_status gm_profile_read(gm_scene* sc, const char* stage, double* total_ms, int64_t* launches)
{
    gm::clear_error();
    if (!sc || !stage) return fail(GM_ERR_INVALID_ARGUMENT, "scene and stage must not be NULL");
    for (int i = 0; i < kStages; ++i) {
        if (std::strcmp(stage, kStageNames[i]) != 0) continue;
        GM_HIP(sc->timers[i].collect());
        if (total_ms) *total_ms = sc->timers[i].total_ms;
        if (launches) *launches = sc->timers[i].launches;
        return GM_OK;
    }
    return fail(GM_ERR_INVALID_ARGUMENT, "unknown stage '%s'", stage);
}

}  // extern "C"
