// zbuffer_api.cpp -- the paper's own visibility approximation (include/gazemap.h,
// gm_render_zbuffers, accumulate_density_zbuffer): per fixation a camera cropped to
// the 4-sigma cone (Sec. 3.3.2, Appendix A), a z-buffer of nearest depths (Sec. 3.2.2)
// cast as one ray per pixel centre over the scene BVH, then the density with the
// frustum filter and the depth test in place of the exact segment test.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gazemap.h"
#include "gm_host.h"
#include "gm_internal.h"

using namespace gm;

namespace {

gm_status check_zparams(gm_scene* sc, const gm_fixations* fix, double theta_deg, const gm_zbuffer_params* zp)
{
    if (!sc) return fail(GM_ERR_INVALID_ARGUMENT, "scene is NULL");
    if (!fix) return fail(GM_ERR_INVALID_ARGUMENT, "fixations is NULL");
    if (fix->n < 0) return fail(GM_ERR_INVALID_ARGUMENT, "fixation count < 0");
    if (fix->n > 0 && (!fix->eye || !fix->gaze || !fix->duration))
        return fail(GM_ERR_INVALID_ARGUMENT, "fixation arrays must not be NULL");
    if (!zp) return fail(GM_ERR_INVALID_ARGUMENT, "z-buffer parameters are NULL");
    if (!(theta_deg > 0.0 && theta_deg <= 10.0))
        return fail(GM_ERR_INVALID_ARGUMENT, "theta_deg must be in (0, 10] for the z-buffer path");
    if (zp->resolution < 8 || zp->resolution > 1024 || zp->resolution % 8)
        return fail(GM_ERR_INVALID_ARGUMENT, "resolution must be a multiple of 8 in [8, 1024]");
    if (!(zp->depth_eps >= 0.0f && zp->depth_eps <= 1.0f))
        return fail(GM_ERR_INVALID_ARGUMENT, "depth_eps must be in [0, 1]");
    if (!(zp->near_plane > 0.0f && zp->far_plane > zp->near_plane && std::isfinite(zp->far_plane)))
        return fail(GM_ERR_INVALID_ARGUMENT, "need 0 < near_plane < far_plane < inf");
    return check_device(sc);
}

// cameras, gate records and the fixed-point scale into w; the buffers into zbuf
gm_status render(gm_scene* sc, DensityWork& w, const gm_fixations* fix, double sigma, const gm_zbuffer_params* zp,
                 float* zbuf, hipStream_t s)
{
    const int32_t F = fix->n;
    GM_HIP(w.fix.ensure(sizeof(FixRec) * (size_t)std::max(F, 1)));
    GM_HIP(w.zcam.ensure(sizeof(ZCam) * (size_t)std::max(F, 1)));
    GM_HIP(w.fx_shift.ensure(16));
    zero(w.fx_shift.p, 16, s);
    launch_zcam_prep(fix->eye, fix->gaze, fix->duration, zp->head, F, sigma, kGateWiden, zp->near_plane,
                     zp->far_plane, w.fix.as<FixRec>(), w.zcam.as<ZCam>(), w.fx_shift.as<int32_t>(), s);
    launch_zbuffer(sc->nodes.as<BvhNode>(), (int64_t)sc->bvh.nodes.size(), sc->tris.as<BvhTri>(),
                   (int64_t)sc->bvh.tris.size(), w.fix.as<FixRec>(), w.zcam.as<ZCam>(), F, zp->resolution, zbuf, s);
    GM_HIP(hipGetLastError());
    return GM_OK;
}

}  // namespace

extern "C" {

gm_status gm_render_zbuffers(gm_scene* sc, const gm_fixations* fix, double theta_deg, const gm_zbuffer_params* zp,
                             float* zbuf, void* stream)
{
    clear_error();
    gm_status st = check_zparams(sc, fix, theta_deg, zp);
    if (st != GM_OK) return st;
    if (fix->n > 0 && !zbuf) return fail(GM_ERR_INVALID_ARGUMENT, "zbuf is NULL");
    const double sigma = std::tan(theta_deg * M_PI / 180.0);
    return render(sc, sc->work, fix, sigma, zp, zbuf, (hipStream_t)stream);
}

gm_status accumulate_density_zbuffer(gm_scene* sc, const float* pos, int64_t n, const gm_fixations* fix,
                                     double theta_deg, const gm_zbuffer_params* zp, float* density,
                                     float* density_norm, float* max_out, void* stream)
{
    clear_error();
    gm_status st = check_zparams(sc, fix, theta_deg, zp);
    if (st != GM_OK) return st;
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GM_ERR_INVALID_ARGUMENT, "n must be in [0, 2^31)");
    if (n > 0 && !pos) return fail(GM_ERR_INVALID_ARGUMENT, "pos is NULL");
    hipStream_t s = (hipStream_t)stream;
    DensityWork& w = sc->work;
    const int32_t F = fix->n;
    const int64_t R = zp->resolution;
    st = density_reserve(w, n, F);
    if (st != GM_OK) return st;
    GM_HIP(w.zbuf.ensure(sizeof(float) * (size_t)std::max<int64_t>(1, (int64_t)F * R * R)));
    const double sigma = std::tan(theta_deg * M_PI / 180.0);
    GM_HIP(sc->tbegin(kStagePrep, s));
    zero(w.stats.p, 8 * kDensityStats, s);
    zero(w.max_acc.p, 8, s);
    st = render(sc, w, fix, sigma, zp, w.zbuf.as<float>(), s);
    if (st != GM_OK) return st;
    density_sort(sc, w, pos, nullptr, nullptr, n, s);
    DensityLaunch a;
    density_args(sc, w, n, F, sigma, GM_OCC_NONE, sc->spl ? sc->spl : 2, 0, a);
    a.zcam = reinterpret_cast<const float*>(w.zcam.p);
    a.zbuf = w.zbuf.as<float>();
    a.zres = (int32_t)R;
    a.zeps = zp->depth_eps;
    GM_HIP(sc->tend(kStagePrep, s));
    if (n > 0 && F > 0) {
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

}  // extern "C"
