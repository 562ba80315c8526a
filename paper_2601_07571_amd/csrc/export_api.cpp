// export_api.cpp -- the export format of Sec. 3.3.3 (include/gazemap.h,
// gm_export_samples): one packed record per sample with its value, object,
// triangle, barycentric coordinates and its position in the object's own frame and
// in the world.
#include <hip/hip_runtime.h>

#include "gazemap.h"
#include "gm_host.h"
#include "gm_internal.h"

using namespace gm;

static_assert(sizeof(gm_export_record) == 48, "export record is 48 bytes");

namespace {

__global__ void k_export(const int32_t* __restrict__ tri, const int32_t* __restrict__ mesh,
                         const float* __restrict__ bary, const float* __restrict__ pos,
                         const float* __restrict__ density, const float* __restrict__ density_norm,
                         const float* __restrict__ pose, const int32_t* __restrict__ tri_mesh,
                         const int64_t* __restrict__ tri_off, int64_t T, int32_t M, int64_t n,
                         gm_export_record* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    gm_export_record r;
    const int32_t t = tri[i];
    const bool tok = t >= 0 && t < T;
    int32_t m = mesh ? mesh[i] : (tok ? tri_mesh[t] : -1);
    if (m < 0 || m >= M) m = -1;
    r.value = density[i];
    r.value_norm = density_norm ? density_norm[i] : __int_as_float(0x7fc00000);
    r.mesh = m;
    r.triangle = (tok && m >= 0 && tri_mesh[t] == m) ? (int32_t)(t - tri_off[m]) : -1;
    r.bary[0] = bary[2 * i];
    r.bary[1] = bary[2 * i + 1];
    const float x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    r.local[0] = x; r.local[1] = y; r.local[2] = z;
    if (pose && m >= 0) {
        const float* P = pose + 12 * (int64_t)m;
        for (int k = 0; k < 3; ++k)
            r.world[k] = (float)((((double)P[4 * k] * x + (double)P[4 * k + 1] * y) + (double)P[4 * k + 2] * z) +
                                 (double)P[4 * k + 3]);
    } else {
        r.world[0] = x; r.world[1] = y; r.world[2] = z;
    }
    out[i] = r;
}

}  // namespace

extern "C" gm_status gm_export_samples(gm_scene* sc, const int32_t* tri, const int32_t* mesh, const float* bary,
                                       const float* pos, const float* density, const float* density_norm,
                                       const float* pose, int64_t n, gm_export_record* out, void* stream)
{
    clear_error();
    if (!sc) return fail(GM_ERR_INVALID_ARGUMENT, "scene is NULL");
    if (n < 0) return fail(GM_ERR_INVALID_ARGUMENT, "n < 0");
    if (n > 0 && (!tri || !bary || !pos || !density || !out))
        return fail(GM_ERR_INVALID_ARGUMENT, "tri, bary, pos, density and out must not be NULL");
    gm_status st = check_device(sc);
    if (st != GM_OK) return st;
    if (n == 0) return GM_OK;
    hipStream_t s = (hipStream_t)stream;
    k_export<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(tri, mesh, bary, pos, density, density_norm, pose,
                                                        sc->tri_mesh.as<int32_t>(), sc->tri_off_d.as<int64_t>(), sc->T,
                                                        sc->M, n, out);
    GM_HIP(hipGetLastError());
    return GM_OK;
}
