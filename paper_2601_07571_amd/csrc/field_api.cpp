// field_api.cpp -- C ABI of the neural density field and of query_density:
// parameter state, the training loop (train kernel, Adam, repacking per step),
// held-out evaluation and the per-mesh gate with the plain fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gazemap.h"
#include "gm_host.h"
#include "gm_internal.h"

using namespace gm;

// One network per mesh, each over its mesh's bounding cube; parameter arrays hold
// the M networks one after the other.
struct gm_field {
    gm_scene* scene = nullptr;
    int32_t M = 0;
    std::vector<FieldGeom> geom;  // [M]
    DevBuf master, m, v, grad, blob, loss;
    DevBuf flag, sel, offs, idx, scan_tmp, pred, l2sums, l2part, geom_d, net_off, net_cnt;
    DevBuf gate_d, need, qoffs, qscan, gpos, gtri, gmesh, gidx, grho, gnorm;
    DevBuf rcnt, rpart, rbase, ridx, take_d;  // routed inference: per-mesh counts, per-chunk counts,
                                              // segment starts, point lists
    DevBuf gpart, lpart;               // training: per-wave gradient and loss slots
    std::vector<float> rel_l2;
    std::vector<uint8_t> gate;
    double norm_max = 0.0;
    double last_loss = NAN;
    int64_t steps = 0;
    bool trained = false;

    ~gm_field()
    {
        for (DevBuf* b : {&master, &m, &v, &grad, &blob, &loss, &flag, &sel, &offs, &idx, &scan_tmp, &pred, &l2sums,
                          &l2part, &geom_d, &net_off, &net_cnt, &gate_d, &need, &qoffs, &qscan, &gpos, &gtri, &gmesh,
                          &gidx, &grho, &gnorm, &rcnt, &rpart, &rbase, &ridx, &take_d, &gpart, &lpart})
            b->release();
    }
};

namespace {

// splitmix64 (Steele, Lea and Flood 2014): the host-side initial weights
uint64_t splitmix64(uint64_t& x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void init_params(uint64_t seed, std::vector<float>& p)
{
    p.assign(kFieldParams, 0.0f);
    uint64_t st = seed;
    auto uni = [&](float lim) { return (float)(((double)(splitmix64(st) >> 11) * 0x1.0p-53 * 2.0 - 1.0) * lim); };
    for (int L = 1; L <= 4; ++L) {
        const int fan_in = L == 1 ? kFieldFeat : kFieldWidth;
        const float lim = (float)std::sqrt(6.0 / fan_in);
        for (int i = 0; i < fan_in * kFieldWidth; ++i) p[(size_t)(kFieldOffW[L] + i)] = uni(lim);
    }
    const float lim5 = (float)std::sqrt(6.0 / kFieldWidth);
    for (int i = 0; i < kFieldWidth; ++i) p[(size_t)(kFieldOffW5 + i)] = uni(lim5);
}

unsigned char* net_blob(gm_field* f, int m) { return f->blob.as<unsigned char>() + (size_t)m * field_pack_bytes(); }

// Adam's bias corrections (Kingma and Ba 2015) for update number `step` (from 1):
// c1 = 1 / (1 - beta1^step), c2 = 1 / (1 - beta2^step), in FP64 then rounded.
void adam_bias_scales(int32_t step, float beta1, float beta2, float& c1, float& c2)
{
    c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
    c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
}

gm_status upload_params(gm_field* f, const float* host, hipStream_t s)
{
    GM_HIP(hipMemcpyAsync(f->master.p, host, sizeof(float) * kFieldParams * (size_t)f->M, hipMemcpyHostToDevice, s));
    launch_field_pack_nets(f->master.as<float>(), f->blob.as<unsigned char>(), f->M, s);
    GM_HIP(hipGetLastError());
    GM_HIP(hipStreamSynchronize(s));
    return GM_OK;
}

FieldRoute route_all() { return FieldRoute{nullptr, nullptr, nullptr, 0, -1}; }

// Every network over its own mesh's points (those of the meshes with take[m] set, NULL:
// all), each point evaluated once, in one launch.
gm_status infer_routed(gm_field* f, const float* pos, int64_t q, float* out, const FieldRoute& route,
                       const uint8_t* take, hipStream_t s)
{
    GM_HIP(f->rcnt.ensure(4 * 3 * (size_t)f->M));
    GM_HIP(f->rbase.ensure(8 * (3 * (size_t)f->M + 1)));
    GM_HIP(f->ridx.ensure(4 * (size_t)field_route_slots(q, f->M)));
    const int64_t pb = field_route_part_bytes(q, f->M);
    if (pb > 0) GM_HIP(f->rpart.ensure((size_t)pb));
    launch_field_infer_routed(f->blob.as<unsigned char>(), (int64_t)field_pack_bytes(), f->geom_d.as<FieldGeom>(),
                              pos, q, out, route, take, f->M, f->rcnt.as<unsigned int>(),
                              pb > 0 ? f->rpart.as<unsigned int>() : nullptr, f->rbase.as<int64_t>(),
                              f->ridx.as<int32_t>(), s);
    GM_HIP(hipGetLastError());
    return GM_OK;
}

}  // namespace

extern "C" {

gm_status gm_field_create(gm_scene* scene, uint64_t seed, double max_cycles, gm_field** out)
{
    clear_error();
    if (!scene || !out) return fail(GM_ERR_INVALID_ARGUMENT, "scene and out must not be NULL");
    *out = nullptr;
    gm_status st = check_device(scene);
    if (st != GM_OK) return st;
    gm_field* f = new (std::nothrow) gm_field();
    if (!f) return fail(GM_ERR_OUT_OF_MEMORY, "host allocation failed");
    f->scene = scene;
    f->M = scene->M;
    // each mesh's bounding box, from the triangle records (vertices in x, y, z order)
    std::vector<float> blo((size_t)(3 * f->M), INFINITY), bhi((size_t)(3 * f->M), -INFINITY);
    for (const BvhTri& r : scene->bvh.tris) {
        if (r.mesh < 0 || r.mesh >= f->M) continue;
        for (int a = 0; a < 3; ++a) {
            const float c[3] = {r.v0[a], r.v1[a], r.v2[a]};
            for (float x : c) {
                blo[(size_t)(3 * r.mesh + a)] = std::min(blo[(size_t)(3 * r.mesh + a)], x);
                bhi[(size_t)(3 * r.mesh + a)] = std::max(bhi[(size_t)(3 * r.mesh + a)], x);
            }
        }
    }
    if (!(max_cycles > 0.0) || !std::isfinite(max_cycles)) max_cycles = 32.0;
    f->geom.resize((size_t)f->M);
    for (int m = 0; m < f->M; ++m) {
        FieldGeom& g = f->geom[(size_t)m];
        float ext = 0.0f;
        for (int a = 0; a < 3; ++a) {
            const bool any = blo[(size_t)(3 * m + a)] <= bhi[(size_t)(3 * m + a)];
            g.lo[a] = any ? blo[(size_t)(3 * m + a)] : 0.0f;
            if (any) ext = std::max(ext, bhi[(size_t)(3 * m + a)] - blo[(size_t)(3 * m + a)]);
        }
        g.inv_ext = ext > 0.0f ? 1.0f / ext : 1.0f;
        for (int b = 0; b < kFieldBands; ++b)
            g.freq[b] = (float)std::pow(max_cycles, (double)b / (double)(kFieldBands - 1));
    }
    f->rel_l2.assign((size_t)scene->M, NAN);
    f->gate.assign((size_t)scene->M, 0);
    hipError_t e = hipSuccess;
    const size_t np = (size_t)kFieldParams * (size_t)f->M;
    for (DevBuf* b : {&f->master, &f->m, &f->v, &f->grad})
        if (e == hipSuccess) e = b->ensure(sizeof(float) * np);
    if (e == hipSuccess) e = f->blob.ensure(field_pack_bytes() * (size_t)f->M);
    if (e == hipSuccess) e = f->loss.ensure(sizeof(double) * (size_t)f->M);
    if (e == hipSuccess) e = f->geom_d.ensure(sizeof(FieldGeom) * (size_t)f->M);
    if (e == hipSuccess)
        e = hipMemcpy(f->geom_d.p, f->geom.data(), sizeof(FieldGeom) * (size_t)f->M, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete f;
        return fail(GM_ERR_OUT_OF_MEMORY, "field allocation: %s", hipGetErrorString(e));
    }
    std::vector<float> p, all;
    for (int m = 0; m < f->M; ++m) {
        init_params(seed + 0x9E3779B97F4A7C15ull * (uint64_t)m, p);
        all.insert(all.end(), p.begin(), p.end());
    }
    st = upload_params(f, all.data(), nullptr);
    if (st != GM_OK) {
        delete f;
        return st;
    }
    zero(f->m.p, sizeof(float) * np, nullptr);
    zero(f->v.p, sizeof(float) * np, nullptr);
    zero(f->grad.p, sizeof(float) * np, nullptr);
    if (hipStreamSynchronize(nullptr) != hipSuccess) {
        delete f;
        return fail(GM_ERR_DEVICE, "field initialisation failed");
    }
    *out = f;
    return GM_OK;
}

gm_status gm_field_destroy(gm_field* f)
{
    clear_error();
    if (f) {
        (void)hipDeviceSynchronize();
        delete f;
    }
    return GM_OK;
}

gm_status gm_field_set_params(gm_field* f, const float* params)
{
    clear_error();
    if (!f || !params) return fail(GM_ERR_INVALID_ARGUMENT, "field and params must not be NULL");
    for (int64_t i = 0; i < (int64_t)kFieldParams * f->M; ++i)
        if (!std::isfinite(params[i])) return fail(GM_ERR_INVALID_ARGUMENT, "parameter %lld is not finite", (long long)i);
    return upload_params(f, params, nullptr);
}

gm_status gm_field_get_params(gm_field* f, float* params)
{
    clear_error();
    if (!f || !params) return fail(GM_ERR_INVALID_ARGUMENT, "field and params must not be NULL");
    GM_HIP(hipDeviceSynchronize());
    GM_HIP(hipMemcpy(params, f->master.p, sizeof(float) * kFieldParams * (size_t)f->M, hipMemcpyDeviceToHost));
    return GM_OK;
}

gm_status gm_field_gradient(gm_field* f, int32_t net, const float* pos, const float* target, int64_t n, float* grad,
                            double* loss)
{
    clear_error();
    if (!f || !pos || !target || !grad || n <= 0 || n > 65536)
        return fail(GM_ERR_INVALID_ARGUMENT, "NULL argument or n outside (0, 65536]");
    if (net < 0 || net >= f->M) return fail(GM_ERR_INVALID_ARGUMENT, "network %d outside [0, %d)", net, f->M);
    gm_status st = check_device(f->scene);
    if (st != GM_OK) return st;
    hipStream_t s = nullptr;
    float* gnet = f->grad.as<float>() + (size_t)net * kFieldParams;
    const int32_t slots = field_train_slots((int32_t)n, 1);
    GM_HIP(f->gpart.ensure(sizeof(float) * kFieldParams * (size_t)slots));
    GM_HIP(f->lpart.ensure(sizeof(double) * (size_t)slots));
    FieldTrain t;
    t.pos = pos;
    t.target = target;
    t.idx = nullptr;
    t.n_idx = n;
    t.batch = (int32_t)n;
    t.inv_batch = (float)(1.0 / (double)n);
    t.key0 = t.key1 = 0;
    t.step = 0;
    t.gpart = f->gpart.as<float>();
    t.lpart = f->lpart.as<double>();
    launch_field_train(net_blob(f, net), f->geom[(size_t)net], t, gnet, f->loss.as<double>(), s);
    GM_HIP(hipGetLastError());
    double l = 0.0;
    GM_HIP(hipMemcpy(grad, gnet, sizeof(float) * kFieldParams, hipMemcpyDeviceToHost));
    GM_HIP(hipMemcpy(&l, f->loss.p, sizeof(double), hipMemcpyDeviceToHost));
    zero(gnet, sizeof(float) * kFieldParams, s);
    GM_HIP(hipStreamSynchronize(s));
    if (loss) *loss = l / (double)n;
    return GM_OK;
}

gm_status gm_debug_adam_step(float* params, float* m, float* v, float* grad, int64_t count, int32_t step, float lr,
                             float beta1, float beta2, float eps, void* stream)
{
    clear_error();
    if (count < 0 || (count > 0 && (!params || !m || !v || !grad)))
        return fail(GM_ERR_INVALID_ARGUMENT, "NULL argument or negative size");
    if (step < 1) return fail(GM_ERR_INVALID_ARGUMENT, "step counts from 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps >= 0.0f && std::isfinite(lr)))
        return fail(GM_ERR_INVALID_ARGUMENT, "beta1, beta2 in [0, 1), eps >= 0, finite lr");
    float c1, c2;
    adam_bias_scales(step, beta1, beta2, c1, c2);
    launch_field_adam(params, m, v, grad, count, lr, beta1, beta2, eps, c1, c2, (hipStream_t)stream);
    GM_HIP(hipGetLastError());
    return GM_OK;
}

gm_status gm_field_train(gm_field* f, const float* pos, const int32_t* mesh, const float* target, int64_t n,
                         const gm_train_params* P, void* stream)
{
    clear_error();
    if (!f || !pos || !mesh || !target || !P) return fail(GM_ERR_INVALID_ARGUMENT, "NULL argument");
    if (n < 2 || n >= ((int64_t)1 << 31)) return fail(GM_ERR_INVALID_ARGUMENT, "n must be in [2, 2^31)");
    if (P->steps < 0 || P->batch < 1 || !(P->lr > 0.0f) || !(P->lr_final >= 0.0f) || !(P->beta1 >= 0.0f) ||
        !(P->beta1 < 1.0f) || !(P->beta2 >= 0.0f) || !(P->beta2 < 1.0f) || !(P->eps > 0.0f) ||
        !(P->holdout > 0.0f) || !(P->holdout < 1.0f) || !(P->max_rel_l2 >= 0.0f))
        return fail(GM_ERR_INVALID_ARGUMENT, "training parameters out of range");
    gm_status st = check_device(f->scene);
    if (st != GM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int32_t M = f->scene->M;
    GM_HIP(f->flag.ensure(4 * (size_t)n));
    GM_HIP(f->sel.ensure(4 * (size_t)n));
    GM_HIP(f->offs.ensure(4 * (size_t)n));
    GM_HIP(f->idx.ensure(4 * (size_t)n));
    GM_HIP(f->scan_tmp.ensure(scan_tmp_bytes(n)));
    GM_HIP(f->pred.ensure(4 * (size_t)n));
    GM_HIP(f->l2sums.ensure(16 * (size_t)M));
    GM_HIP(f->l2part.ensure((size_t)field_l2_part_bytes(n, M)));

    // held-out split (one Philox draw per point, for every network)
    const uint32_t key0 = (uint32_t)P->seed, key1 = (uint32_t)(P->seed >> 32);
    const uint32_t thr = (uint32_t)std::min(4294967295.0, std::floor((double)P->holdout * 4294967296.0));
    launch_field_split(n, key0, key1, thr, f->flag.as<uint32_t>(), s);
    const size_t np = (size_t)kFieldParams * (size_t)M;
    zero(f->m.p, sizeof(float) * np, s);
    zero(f->v.p, sizeof(float) * np, s);
    zero(f->grad.p, sizeof(float) * np, s);
    zero(f->pred.p, 4 * (size_t)n, s);
    double last = NAN;
    std::vector<uint8_t> has_train((size_t)M, 0);
    // each mesh's training points, compacted one mesh after the other into idx
    std::vector<int64_t> off((size_t)M, 0), cnt((size_t)M, 0);
    int64_t total = 0;
    for (int32_t net = 0; net < M; ++net) {
        launch_field_select(f->flag.as<uint32_t>(), mesh, net, n, f->sel.as<uint32_t>(), s);
        launch_exclusive_scan_u32(f->sel.as<uint32_t>(), f->offs.as<uint32_t>(), n, f->scan_tmp.p, s);
        launch_field_compact(f->sel.as<uint32_t>(), f->offs.as<uint32_t>(), n, f->idx.as<int32_t>() + total, s);
        uint32_t last_off = 0, last_sel = 0;
        GM_HIP(hipMemcpyAsync(&last_off, f->offs.as<uint32_t>() + (n - 1), 4, hipMemcpyDeviceToHost, s));
        GM_HIP(hipMemcpyAsync(&last_sel, f->sel.as<uint32_t>() + (n - 1), 4, hipMemcpyDeviceToHost, s));
        GM_HIP(hipStreamSynchronize(s));
        off[(size_t)net] = total;
        cnt[(size_t)net] = (int64_t)last_off + last_sel;
        total += cnt[(size_t)net];
        has_train[(size_t)net] = cnt[(size_t)net] > 0;  // a mesh without training points keeps its gate closed
    }
    GM_HIP(f->net_off.ensure(sizeof(int64_t) * (size_t)M));
    GM_HIP(f->net_cnt.ensure(sizeof(int64_t) * (size_t)M));
    GM_HIP(hipMemcpyAsync(f->net_off.p, off.data(), sizeof(int64_t) * (size_t)M, hipMemcpyHostToDevice, s));
    GM_HIP(hipMemcpyAsync(f->net_cnt.p, cnt.data(), sizeof(int64_t) * (size_t)M, hipMemcpyHostToDevice, s));
    FieldNets nets;
    nets.geom = f->geom_d.as<FieldGeom>();
    nets.off = f->net_off.as<int64_t>();
    nets.cnt = f->net_cnt.as<int64_t>();
    nets.pack_stride = (int64_t)field_pack_bytes();
    // every network takes the same steps at once: one launch per step for all of them
    // (network m draws its batches with key0 ^ m, as a launch of its own would)
    FieldTrain t;
    t.pos = pos;
    t.target = target;
    t.idx = f->idx.as<int32_t>();
    t.n_idx = 0;
    t.batch = P->batch;
    t.inv_batch = 1.0f / (float)P->batch;
    t.key0 = key0 ^ 0x5bd1e995u;
    t.key1 = key1 ^ 0x1b873593u;
    const int32_t slots = field_train_slots(P->batch, M);
    GM_HIP(f->gpart.ensure(sizeof(float) * kFieldParams * (size_t)slots * (size_t)M));
    GM_HIP(f->lpart.ensure(sizeof(double) * (size_t)slots * (size_t)M));
    t.gpart = f->gpart.as<float>();
    t.lpart = f->lpart.as<double>();
    for (int32_t it = 0; it < P->steps && total > 0; ++it) {
        t.step = (uint32_t)it;
        launch_field_train_nets(f->blob.as<unsigned char>(), nets, M, t, f->grad.as<float>(), f->loss.as<double>(), s);
        const double frac = P->steps > 1 ? (double)it / (double)(P->steps - 1) : 1.0;
        const double lr = P->lr_final + 0.5 * (P->lr - P->lr_final) * (1.0 + std::cos(M_PI * frac));
        float c1, c2;
        adam_bias_scales(it + 1, P->beta1, P->beta2, c1, c2);
        launch_field_adam(f->master.as<float>(), f->m.as<float>(), f->v.as<float>(), f->grad.as<float>(),
                          (int64_t)M * kFieldParams, (float)lr, P->beta1, P->beta2, P->eps, c1, c2, s);
        launch_field_pack_nets(f->master.as<float>(), f->blob.as<unsigned char>(), M, s);
    }
    GM_HIP(hipGetLastError());
    if (P->steps > 0 && total > 0) {
        std::vector<double> l((size_t)M, NAN);
        GM_HIP(hipMemcpyAsync(l.data(), f->loss.p, sizeof(double) * (size_t)M, hipMemcpyDeviceToHost, s));
        GM_HIP(hipStreamSynchronize(s));
        for (int32_t net = 0; net < M; ++net)
            if (has_train[(size_t)net]) last = std::isnan(last) ? l[(size_t)net] : std::max(last, l[(size_t)net]);
    }
    // each network's values at its mesh's points, for the held-out error
    GM_HIP(f->take_d.ensure((size_t)M));
    GM_HIP(hipMemcpyAsync(f->take_d.p, has_train.data(), (size_t)M, hipMemcpyHostToDevice, s));
    {
        gm_status rs = infer_routed(f, pos, n, f->pred.as<float>(), FieldRoute{mesh, nullptr, nullptr, 0, -1},
                                    f->take_d.as<uint8_t>(), s);
        if (rs != GM_OK) return rs;
    }

    // held-out relative L2 per mesh
    launch_field_l2(f->pred.as<float>(), target, mesh, f->flag.as<uint32_t>(), n, M, f->l2part.as<double>(),
                    f->l2sums.as<double>(), s);
    GM_HIP(hipGetLastError());
    std::vector<double> sums((size_t)(2 * M));
    GM_HIP(hipMemcpyAsync(sums.data(), f->l2sums.p, 16 * (size_t)M, hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    f->last_loss = P->steps > 0 ? last / (double)P->batch : NAN;
    f->steps = P->steps;
    f->norm_max = P->target_max;
    f->trained = true;
    for (int32_t m = 0; m < M; ++m) {
        const double d2 = sums[(size_t)(2 * m)], t2 = sums[(size_t)(2 * m + 1)];
        double rel = NAN;
        if (t2 > 0.0) rel = std::sqrt(d2 / t2);
        else if (d2 == 0.0 && t2 == 0.0) rel = NAN;  // no held-out point of this mesh
        f->rel_l2[(size_t)m] = (float)rel;
        f->gate[(size_t)m] =
            (has_train[(size_t)m] && std::isfinite(rel) && rel <= P->max_rel_l2 && std::isfinite(f->last_loss)) ? 1 : 0;
    }
    GM_HIP(f->gate_d.ensure((size_t)M));
    GM_HIP(hipMemcpy(f->gate_d.p, f->gate.data(), (size_t)M, hipMemcpyHostToDevice));
    return GM_OK;
}

gm_status gm_field_predict(gm_field* f, const float* pos, const int32_t* mesh, int64_t q, float* out, void* stream)
{
    clear_error();
    if (!f || q < 0 || q >= ((int64_t)1 << 31) || (q > 0 && (!pos || !out)))
        return fail(GM_ERR_INVALID_ARGUMENT, "NULL argument or q outside [0, 2^31)");
    if (!mesh && f->M > 1) return fail(GM_ERR_INVALID_ARGUMENT, "mesh is required with more than one mesh");
    gm_status st = check_device(f->scene);
    if (st != GM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (!mesh) {
        launch_field_infer(net_blob(f, 0), f->geom[0], pos, q, out, route_all(), s);
        GM_HIP(hipGetLastError());
        return GM_OK;
    }
    return infer_routed(f, pos, q, out, FieldRoute{mesh, nullptr, nullptr, 0, -1}, nullptr, s);
}

gm_status gm_field_info(gm_field* f, float* rel_l2, uint8_t* gate, double* loss, int64_t* steps)
{
    clear_error();
    if (!f) return fail(GM_ERR_INVALID_ARGUMENT, "field is NULL");
    if (rel_l2) std::memcpy(rel_l2, f->rel_l2.data(), sizeof(float) * f->rel_l2.size());
    if (gate) std::memcpy(gate, f->gate.data(), f->gate.size());
    if (loss) *loss = f->last_loss;
    if (steps) *steps = f->steps;
    return GM_OK;
}

gm_status query_density(gm_field* f, gm_scene* sc, const gm_fixations* fix, double theta_deg, uint32_t flags,
                        const float* pos, const int32_t* tri, const int32_t* mesh, int64_t q, double ref_max,
                        float* out, uint8_t* used_fallback, void* stream)
{
    clear_error();
    if (!sc || !fix) return fail(GM_ERR_INVALID_ARGUMENT, "scene and fixations must not be NULL");
    if (f && f->scene != sc) return fail(GM_ERR_INVALID_ARGUMENT, "field belongs to another scene");
    if (q < 0 || q >= ((int64_t)1 << 31)) return fail(GM_ERR_INVALID_ARGUMENT, "q must be in [0, 2^31)");
    if (q > 0 && (!pos || !out)) return fail(GM_ERR_INVALID_ARGUMENT, "pos and out must not be NULL");
    if (!(theta_deg > 0.0 && theta_deg < 45.0)) return fail(GM_ERR_INVALID_ARGUMENT, "theta_deg must be in (0, 45)");
    if ((flags & GM_OCC_MASK) > GM_OCC_FULL || (flags & ~GM_OCC_MASK))
        return fail(GM_ERR_INVALID_ARGUMENT, "unknown flags 0x%x", flags);
    gm_status st = check_device(sc);
    if (st != GM_OK) return st;
    if (q == 0) return GM_OK;
    hipStream_t s = (hipStream_t)stream;
    const bool use_field = f && f->trained;
    if (use_field && (mesh || tri)) {
        bool any = false;
        for (uint8_t g : f->gate) any = any || g;
        if (any) {
            st = infer_routed(f, pos, q, out, FieldRoute{mesh, tri, sc->tri_mesh.as<int32_t>(), sc->T, -1},
                              f->gate_d.as<uint8_t>(), s);
            if (st != GM_OK) return st;
        }
    }
    // scratch lives in the field when there is one, else in per-call buffers
    DevBuf local_need, local_offs, local_scan;
    DevBuf& need = f ? f->need : local_need;
    DevBuf& offs = f ? f->qoffs : local_offs;
    DevBuf& scan = f ? f->qscan : local_scan;
    GM_HIP(need.ensure(4 * (size_t)q));
    GM_HIP(offs.ensure(4 * (size_t)q));
    GM_HIP(scan.ensure(scan_tmp_bytes(q)));
    launch_gate_flags(mesh, tri, sc->tri_mesh.as<int32_t>(), sc->T, use_field ? f->gate_d.as<uint8_t>() : nullptr,
                      sc->M, q, need.as<uint32_t>(), s);
    if (used_fallback) launch_used_flags(need.as<uint32_t>(), q, used_fallback, s);
    launch_exclusive_scan_u32(need.as<uint32_t>(), offs.as<uint32_t>(), q, scan.p, s);
    uint32_t last_off = 0, last_need = 0;
    GM_HIP(hipMemcpyAsync(&last_off, offs.as<uint32_t>() + (q - 1), 4, hipMemcpyDeviceToHost, s));
    GM_HIP(hipMemcpyAsync(&last_need, need.as<uint32_t>() + (q - 1), 4, hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    const int64_t m = (int64_t)last_off + last_need;
    if (m == 0) return GM_OK;

    DevBuf lg[6];
    DevBuf& gpos = f ? f->gpos : lg[0];
    DevBuf& gtri = f ? f->gtri : lg[1];
    DevBuf& gmesh = f ? f->gmesh : lg[2];
    DevBuf& gidx = f ? f->gidx : lg[3];
    DevBuf& grho = f ? f->grho : lg[4];
    DevBuf& gnorm = f ? f->gnorm : lg[5];
    GM_HIP(gpos.ensure(12 * (size_t)m));
    GM_HIP(gtri.ensure(4 * (size_t)m));
    GM_HIP(gmesh.ensure(4 * (size_t)m));
    GM_HIP(gidx.ensure(4 * (size_t)m));
    GM_HIP(grho.ensure(4 * (size_t)m));
    GM_HIP(gnorm.ensure(16));
    launch_gather_points(pos, tri, mesh, need.as<uint32_t>(), offs.as<uint32_t>(), q, gpos.as<float>(),
                         gtri.as<int32_t>(), gmesh.as<int32_t>(), gidx.as<int32_t>(), s);
    GM_HIP(hipGetLastError());
    st = accumulate_density(sc, gpos.as<float>(), tri ? gtri.as<int32_t>() : nullptr,
                            mesh ? gmesh.as<int32_t>() : nullptr, m, fix, theta_deg, flags, grho.as<float>(), nullptr,
                            gnorm.as<float>(), stream);
    if (st != GM_OK) return st;
    double norm = ref_max > 0.0 ? ref_max : (f && f->norm_max > 0.0 ? f->norm_max : 0.0);
    if (norm > 0.0) {
        const float nf = (float)norm;
        uint32_t bits;
        std::memcpy(&bits, &nf, 4);
        fill_u32(gnorm.p, 1, bits, s);
    }
    launch_scatter_fallback(grho.as<float>(), gidx.as<int32_t>(), m, gnorm.as<float>(), out, s);
    GM_HIP(hipGetLastError());
    if (!f) GM_HIP(hipStreamSynchronize(s));  // per-call scratch is freed on return
    return GM_OK;
}

}  // extern "C"
