// batch_api.cpp -- many density maps (recording sessions of uneven size, each with
// its own meshes, fixations and angular deviation) in one persistent launch:
// per-session preparation, one work queue of (session, tile, fixation chunk)
// items sorted longest first, per-session normalisation; the whole sequence is
// captured once in a HIP graph and replayed by gm_batch_run.  The tile shape
// (samples per lane), the LDS fixation block and the chunk length come from an
// autotuner that times candidates on the batch itself and keeps the winner in a
// JSON cache keyed by the batch's shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "gazemap.h"
#include "gm_host.h"
#include "gm_internal.h"

using namespace gm;

namespace {

struct TileConfig {
    int spl = 2;
    int fb = 128;
    int chunk = 0;  // fixations per work item (0: automatic per session)
};

}  // namespace

struct gm_batch {
    std::vector<gm_session> sessions;
    std::vector<std::unique_ptr<DensityWork>> work;
    std::vector<DensityLaunch> launches;
    std::vector<int4> items;
    DevBuf d_launches, d_items, d_head;
    TileConfig cfg;
    int grid = 0;
    double tune_ms = -1.0;
    int from_cache = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~gm_batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace {

int ilog2(double v) { return v >= 1.0 ? (int)std::floor(std::log2(v)) : 0; }

std::string shape_key(const gm_batch* b)
{
    double N = 0, F = 0, P = 0, occ = 0, th = 0;
    for (const gm_session& s : b->sessions) {
        N += (double)s.n;
        F += (double)s.fix.n;
        P += (double)s.n * (double)s.fix.n;
        occ = std::max(occ, (double)(s.flags & GM_OCC_MASK));
        th += s.theta_deg;
    }
    char buf[160];
    std::snprintf(buf, sizeof(buf), "gfx950/S%zu/N%d/F%d/P%d/occ%d/th%d", b->sessions.size(), ilog2(N), ilog2(F),
                  ilog2(P), (int)occ, (int)std::lround(th / std::max<size_t>(1, b->sessions.size()) * 4.0));
    return buf;
}

// The cache is a JSON object {"<key>": {"spl": s, "fb": f, "chunk": c, "ms": t}, ...},
// one entry per line as written by save_cache.
bool load_cache(const char* path, const std::string& key, TileConfig& cfg, double& ms)
{
    if (!path || !*path) return false;
    FILE* fp = std::fopen(path, "r");
    if (!fp) return false;
    char line[512];
    bool found = false;
    const std::string want = "\"" + key + "\"";
    while (std::fgets(line, sizeof(line), fp)) {
        const char* k = std::strstr(line, want.c_str());
        if (!k) continue;
        int spl = 0, fb = 0, chunk = 0;
        double t = 0;
        const char* v = std::strchr(k + want.size(), '{');
        if (v && std::sscanf(v, "{\"spl\": %d, \"fb\": %d, \"chunk\": %d, \"ms\": %lf", &spl, &fb, &chunk, &t) == 4 &&
            (spl == 1 || spl == 2 || spl == 4) && (fb == 64 || fb == 128 || fb == 256) && chunk >= 0) {
            cfg.spl = spl;
            cfg.fb = fb;
            cfg.chunk = chunk;
            ms = t;
            found = true;
        }
    }
    std::fclose(fp);
    return found;
}

void save_cache(const char* path, const std::string& key, const TileConfig& cfg, double ms)
{
    if (!path || !*path) return;
    std::vector<std::string> keep;
    if (FILE* fp = std::fopen(path, "r")) {
        char line[512];
        while (std::fgets(line, sizeof(line), fp)) {
            std::string l(line);
            if (l.find("\"spl\"") == std::string::npos) continue;
            if (l.find("\"" + key + "\"") != std::string::npos) continue;
            while (!l.empty() && (l.back() == '\n' || l.back() == ',' || l.back() == ' ')) l.pop_back();
            keep.push_back(l);
        }
        std::fclose(fp);
    }
    char buf[400];
    std::snprintf(buf, sizeof(buf), "  \"%s\": {\"spl\": %d, \"fb\": %d, \"chunk\": %d, \"ms\": %.4f}", key.c_str(),
                  cfg.spl, cfg.fb, cfg.chunk, ms);
    keep.push_back(buf);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return;
    std::fprintf(fp, "{\n");
    for (size_t i = 0; i < keep.size(); ++i) std::fprintf(fp, "%s%s\n", keep[i].c_str(), i + 1 < keep.size() ? "," : "");
    std::fprintf(fp, "}\n");
    std::fclose(fp);
    std::rename(tmp.c_str(), path);
}

// per-session preparation (kernels queued on s) and the sorted work queue
gm_status prepare(gm_batch* b, const TileConfig& cfg, hipStream_t s)
{
    b->launches.resize(b->sessions.size());
    b->items.clear();
    std::vector<double> cost;
    for (size_t i = 0; i < b->sessions.size(); ++i) {
        const gm_session& ss = b->sessions[i];
        gm_status st = density_prep(ss.scene, *b->work[i], ss.pos, ss.tri, ss.mesh, ss.n, &ss.fix, ss.theta_deg,
                                    ss.flags & GM_OCC_MASK, cfg.spl, cfg.chunk, b->launches[i], s);
        if (st != GM_OK) return st;
        const DensityLaunch& a = b->launches[i];
        if (ss.n == 0 || ss.fix.n == 0) continue;
        const int64_t per_tile = 256 * cfg.spl;
        const int64_t tiles = (ss.n + per_tile - 1) / per_tile;
        const double sig = std::tan(ss.theta_deg * M_PI / 180.0);
        for (int64_t t = 0; t < tiles; ++t)
            for (int c = 0; c < a.n_chunks; ++c) {
                const double ns = (double)std::min(per_tile, ss.n - t * per_tile);
                const double nf = (double)std::min(a.fix_per_chunk, ss.fix.n - c * a.fix_per_chunk);
                // pairs, weighted up for the larger cone (more exact evaluations and rays)
                cost.push_back(ns * nf * (1.0 + 4000.0 * sig * sig));
                b->items.push_back(make_int4((int)i, (int)t, c, 0));
            }
    }
    std::vector<size_t> order(b->items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    std::vector<int4> sorted(order.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = b->items[order[i]];
    b->items.swap(sorted);
    return GM_OK;
}

gm_status upload_plan(gm_batch* b, hipStream_t s)
{
    GM_HIP(b->d_launches.ensure(sizeof(DensityLaunch) * std::max<size_t>(1, b->launches.size())));
    GM_HIP(b->d_items.ensure(sizeof(int4) * std::max<size_t>(1, b->items.size())));
    GM_HIP(b->d_head.ensure(16));
    GM_HIP(hipMemcpyAsync(b->d_launches.p, b->launches.data(), sizeof(DensityLaunch) * b->launches.size(),
                          hipMemcpyHostToDevice, s));
    if (!b->items.empty())
        GM_HIP(hipMemcpyAsync(b->d_items.p, b->items.data(), sizeof(int4) * b->items.size(), hipMemcpyHostToDevice, s));
    GM_HIP(hipStreamSynchronize(s));
    return GM_OK;
}

void launch_queue(gm_batch* b, const TileConfig& cfg, hipStream_t s)
{
    zero(b->d_head.p, 16, s);
    launch_density_queue(b->d_launches.as<DensityLaunch>(), b->d_items.as<int4>(), (int32_t)b->items.size(),
                         b->d_head.as<unsigned int>(), cfg.spl, cfg.fb, b->grid, s);
}

gm_status finalize_all(gm_batch* b, hipStream_t s)
{
    for (size_t i = 0; i < b->sessions.size(); ++i) {
        const gm_session& ss = b->sessions[i];
        gm_status st = density_finalize(*b->work[i], ss.n, ss.density, ss.density_norm, ss.max_out, s);
        if (st != GM_OK) return st;
    }
    return GM_OK;
}

// time one candidate: preparation, queue kernel (timed), finalisation
gm_status time_config(gm_batch* b, const TileConfig& cfg, hipStream_t s, double& ms)
{
    gm_status st = prepare(b, cfg, s);
    if (st != GM_OK) return st;
    st = upload_plan(b, s);
    if (st != GM_OK) return st;
    hipEvent_t e0, e1;
    GM_HIP(hipEventCreate(&e0));
    GM_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
        if (rep > 0) {
            st = prepare(b, cfg, s);
            if (st != GM_OK) return st;
        }
        (void)hipEventRecord(e0, s);
        launch_queue(b, cfg, s);
        (void)hipEventRecord(e1, s);
        hipError_t e = hipEventSynchronize(e1);
        if (e != hipSuccess) return fail(GM_ERR_DEVICE, "autotune: %s", hipGetErrorString(e));
        float t = 0.0f;
        (void)hipEventElapsedTime(&t, e0, e1);
        best = std::min(best, t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ms = best;
    return GM_OK;
}

}  // namespace

extern "C" {

gm_status gm_batch_create(const gm_session* sessions, int32_t n_sessions, const char* tune_cache, int32_t tune,
                          gm_batch** out, void* stream)
{
    clear_error();
    if (!out) return fail(GM_ERR_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    if (!sessions || n_sessions < 1 || n_sessions > 65536)
        return fail(GM_ERR_INVALID_ARGUMENT, "n_sessions must be in [1, 65536]");
    for (int32_t i = 0; i < n_sessions; ++i) {
        const gm_session& s = sessions[i];
        gm_status st = check_density_args(s.scene, s.pos, s.n, &s.fix, s.theta_deg, s.flags);
        if (st != GM_OK) return fail(st, "session %d: %s", i, last_error());
    }
    std::unique_ptr<gm_batch> b(new (std::nothrow) gm_batch());
    if (!b) return fail(GM_ERR_OUT_OF_MEMORY, "host allocation failed");
    b->sessions.assign(sessions, sessions + n_sessions);
    for (int32_t i = 0; i < n_sessions; ++i) {
        b->work.emplace_back(new DensityWork());
        gm_status st = density_reserve(*b->work.back(), sessions[i].n, sessions[i].fix.n);
        if (st != GM_OK) return st;
    }
    hipStream_t s = (hipStream_t)stream;
    if (!tune_cache || !*tune_cache) tune_cache = std::getenv("GM_TUNE_CACHE");
    const std::string key = shape_key(b.get());
    TileConfig cfg;
    double ms = -1.0;
    const bool cached = tune == 0 && load_cache(tune_cache, key, cfg, ms);
    b->grid = density_queue_grid(cfg.spl, cfg.fb);
    if (cached) {
        b->from_cache = 1;
    } else if (tune) {
        // coordinate search: samples per lane, then the LDS fixation block, then the chunk length
        TileConfig best = cfg, c = cfg;
        double best_ms = 1e30, t = 0;
        for (int spl : {1, 2, 4}) {
            c.spl = spl;
            b->grid = density_queue_grid(c.spl, c.fb);
            gm_status st = time_config(b.get(), c, s, t);
            if (st != GM_OK) return st;
            if (t < best_ms) { best_ms = t; best = c; }
        }
        c = best;
        for (int fb : {64, 256}) {
            c.fb = fb;
            b->grid = density_queue_grid(c.spl, c.fb);
            gm_status st = time_config(b.get(), c, s, t);
            if (st != GM_OK) return st;
            if (t < best_ms) { best_ms = t; best = c; }
        }
        c = best;
        for (int chunk : {256, 1024, 4096}) {
            c.chunk = chunk;
            b->grid = density_queue_grid(c.spl, c.fb);
            gm_status st = time_config(b.get(), c, s, t);
            if (st != GM_OK) return st;
            if (t < best_ms) { best_ms = t; best = c; }
        }
        cfg = best;
        ms = best_ms;
        save_cache(tune_cache, key, cfg, ms);
    }
    b->cfg = cfg;
    b->tune_ms = ms;
    b->grid = density_queue_grid(cfg.spl, cfg.fb);

    // the plan for the chosen configuration, then the captured graph
    gm_status st = prepare(b.get(), cfg, s);
    if (st != GM_OK) return st;
    st = upload_plan(b.get(), s);
    if (st != GM_OK) return st;
    GM_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    GM_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    st = prepare(b.get(), cfg, b->cap);
    if (st == GM_OK) {
        launch_queue(b.get(), cfg, b->cap);
        st = finalize_all(b.get(), b->cap);
    }
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->cap, &g);
    if (st != GM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (ce != hipSuccess) return fail(GM_ERR_DEVICE, "graph capture: %s", hipGetErrorString(ce));
    b->graph = g;
    GM_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    *out = b.release();
    return GM_OK;
}

gm_status gm_batch_run(gm_batch* b, void* stream)
{
    clear_error();
    if (!b || !b->exec) return fail(GM_ERR_INVALID_ARGUMENT, "batch is NULL or not planned");
    GM_HIP(hipGraphLaunch(b->exec, (hipStream_t)stream));
    return GM_OK;
}

gm_status gm_batch_info(const gm_batch* b, int32_t* samples_per_lane, int32_t* fix_block, int32_t* fix_per_chunk,
                        int64_t* work_items, double* tuned_ms, int32_t* from_cache)
{
    clear_error();
    if (!b) return fail(GM_ERR_INVALID_ARGUMENT, "batch is NULL");
    if (samples_per_lane) *samples_per_lane = b->cfg.spl;
    if (fix_block) *fix_block = b->cfg.fb;
    if (fix_per_chunk) *fix_per_chunk = b->cfg.chunk;
    if (work_items) *work_items = (int64_t)b->items.size();
    if (tuned_ms) *tuned_ms = b->tune_ms;
    if (from_cache) *from_cache = b->from_cache;
    return GM_OK;
}

gm_status gm_batch_destroy(gm_batch* b)
{
    clear_error();
    if (b) {
        (void)hipDeviceSynchronize();
        delete b;
    }
    return GM_OK;
}

}  // extern "C"
