// k_sampler.hip -- area weights, per-mesh counts and the area-weighted Philox
// sampler (Sec. 3.1: sample density in samples per square metre, independent of
// the triangulation), and the paper's per-triangle lattice sampler.  Built with -ffp-contract=off: every FP64 expression below
// is evaluated as written, one IEEE round-to-nearest operation at a time, so the
// sample positions are reproducible bit for bit from the definition.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gm_internal.h"
#include "gm_philox.h"

namespace gm {
namespace {

constexpr int kBlock = 256;

// Half the norm of the edge cross product, FP64, fixed order (the area that sets
// the sample share of a triangle).
__global__ void k_tri_area(const float* __restrict__ V, const int32_t* __restrict__ I,
                           const int32_t* __restrict__ tri_mesh, int64_t T, double* __restrict__ area,
                           unsigned long long* __restrict__ max_bits)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool live = t < T;
    const int64_t tt = live ? t : T - 1;
    const int32_t i0 = I[3 * tt], i1 = I[3 * tt + 1], i2 = I[3 * tt + 2];
    const double ax = V[3 * i0], ay = V[3 * i0 + 1], az = V[3 * i0 + 2];
    const double ux = (double)V[3 * i1] - ax, uy = (double)V[3 * i1 + 1] - ay, uz = (double)V[3 * i1 + 2] - az;
    const double wx = (double)V[3 * i2] - ax, wy = (double)V[3 * i2 + 1] - ay, wz = (double)V[3 * i2 + 2] - az;
    const double cx = uy * wz - uz * wy;
    const double cy = uz * wx - ux * wz;
    const double cz = ux * wy - uy * wx;
    double sq = cx * cx + cy * cy;
    sq = sq + cz * cz;
    const double a = 0.5 * sqrt(sq);
    if (live) area[t] = a;
    // Per-mesh maximum.  Non-negative doubles order like their bit patterns, so the
    // maximum is an integer maximum; reduce across the wave first when the whole
    // wave lies in one mesh (all but a few waves), else one atomic per lane.
    const int mesh = tri_mesh[tt];
    unsigned long long bits = live ? (unsigned long long)__double_as_longlong(a) : 0ull;
    const int mesh0 = __builtin_amdgcn_readfirstlane(mesh);
    if (__ballot(mesh != mesh0) == 0) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) bits = max(bits, (unsigned long long)__shfl_xor(bits, d, 64));
        if ((threadIdx.x & 63) == 0) atomicMax(&max_bits[mesh0], bits);
    } else if (live) {
        atomicMax(&max_bits[mesh], bits);
    }
}

// S_m = 52 - e with T_m * max A = f 2^e, f in [0.5, 1): the mesh total of the
// fixed-point weights then stays below 2^52.
__global__ void k_mesh_scale(const unsigned long long* __restrict__ max_bits, const int64_t* __restrict__ tri_off,
                             int32_t M, int32_t* __restrict__ S)
{
    const int m = blockIdx.x * kBlock + threadIdx.x;
    if (m >= M) return;
    const double mx = __longlong_as_double((long long)max_bits[m]);
    int e = 0;
    if (mx > 0.0) {
        (void)frexp((double)(tri_off[m + 1] - tri_off[m]) * mx, &e);
        S[m] = 52 - e;
    } else {
        S[m] = 0;
    }
}

__global__ void k_tri_weight(const double* __restrict__ area, const int32_t* __restrict__ tri_mesh,
                             const int32_t* __restrict__ S, int64_t T, unsigned long long* __restrict__ W)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= T) return;
    W[t] = (unsigned long long)floor(ldexp(area[t], S[tri_mesh[t]]));
}

// One thread: per-mesh totals from the global inclusive scan, counts
// round(k * total 2^-S) and sample offsets.  M is at most 4096.
__global__ void k_mesh_counts(const unsigned long long* __restrict__ C, const int64_t* __restrict__ tri_off,
                              const int32_t* __restrict__ S, int32_t M, double k, int64_t* __restrict__ counts,
                              int64_t* __restrict__ offsets, unsigned long long* __restrict__ mesh_total)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t run = 0;
    for (int32_t m = 0; m < M; ++m) {
        const int64_t a = tri_off[m], b = tri_off[m + 1];
        const unsigned long long base = a > 0 ? C[a - 1] : 0ull;
        const unsigned long long tot = C[b - 1] - base;
        const double area = ldexp((double)tot, -S[m]);
        const int64_t n = tot ? (int64_t)floor(area * k + 0.5) : 0;
        counts[m] = n;
        offsets[m] = run;
        mesh_total[m] = tot;
        run += n;
    }
    offsets[M] = run;
}

// The guide table: for bucket k of mesh m (targets k 2^gsh .. (k + 1) 2^gsh - 1), the
// triangle that its lowest target selects, found by the full binary search; the closing
// entry of each mesh is its last triangle.  Selection is monotone in the target, so every
// target of bucket k selects a triangle between guide[k] and guide[k + 1].
__global__ void k_sample_guide(const unsigned long long* __restrict__ C, const int64_t* __restrict__ tri_off,
                               const int64_t* __restrict__ goff, const int32_t* __restrict__ gsh, int32_t M,
                               int64_t G, int32_t* __restrict__ guide)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= G) return;
    int32_t lo = 0, hi = M - 1;  // last m with goff[m] <= e
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (goff[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int32_t m = lo;
    const int64_t a = tri_off[m], b = tri_off[m + 1];
    if (b <= a) return;
    const int64_t k = e - goff[m];
    if (e == goff[m + 1] - 1) {  // closing entry
        guide[e] = (int32_t)(b - 1);
        return;
    }
    const unsigned long long goal = (a > 0 ? C[a - 1] : 0ull) + ((unsigned long long)k << gsh[m]);
    int64_t l = a, h = b - 1;
    while (l < h) {
        const int64_t mid = l + ((h - l) >> 1);
        if (C[mid] > goal) h = mid; else l = mid + 1;
    }
    guide[e] = (int32_t)l;
}

__global__ void __launch_bounds__(kBlock)
k_sample(const float* __restrict__ V, const int32_t* __restrict__ I, const unsigned long long* __restrict__ C,
         const int64_t* __restrict__ tri_off, const int64_t* __restrict__ offsets,
         const unsigned long long* __restrict__ mesh_total, const int32_t* __restrict__ guide,
         const int64_t* __restrict__ goff, const int32_t* __restrict__ gsh, int32_t M, int64_t N, uint32_t key0,
         uint32_t key1, int32_t* __restrict__ tri_out, int32_t* __restrict__ mesh_out, float* __restrict__ bary_out,
         float* __restrict__ pos_out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    // mesh of sample i: last m with offsets[m] <= i (offsets is non-decreasing)
    int32_t lo = 0, hi = M - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (offsets[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const int32_t m = lo;
    const uint64_t j = (uint64_t)(i - offsets[m]);
    uint32_t x0 = (uint32_t)j, x1 = (uint32_t)(j >> 32), x2 = (uint32_t)m, x3 = 0u;
    philox4x32_10(x0, x1, x2, x3, key0, key1);

    // area-weighted triangle: the first with inclusive weight sum above the target
    const uint64_t U = ((uint64_t)x0 << 32) | (uint64_t)x1;
    const uint64_t target = __umul64hi(U, mesh_total[m]);
    const int64_t a = tri_off[m];
    const uint64_t goal = (a > 0 ? C[a - 1] : 0ull) + target;
    // the guide bucket bounds the search (usually to one or two triangles)
    const int64_t gk = goff[m] + (int64_t)(target >> gsh[m]);
    int64_t l = guide[gk], h = guide[gk + 1];
    while (l < h) {
        const int64_t mid = l + ((h - l) >> 1);
        if (C[mid] > goal) h = mid; else l = mid + 1;
    }
    const int64_t t = l;

    // uniform point in the triangle by the square-root warp
    const double u = ldexp((double)x2, -32);
    const double v = ldexp((double)x3, -32);
    const double su = sqrt(u);
    const double b1 = su * (1.0 - v);
    const double b2 = su * v;
    const double b0 = 1.0 - su;
    const int32_t i0 = I[3 * t], i1 = I[3 * t + 1], i2 = I[3 * t + 2];
    if (tri_out) tri_out[i] = (int32_t)t;
    if (mesh_out) mesh_out[i] = m;
    if (bary_out) {
        bary_out[2 * i] = (float)b1;
        bary_out[2 * i + 1] = (float)b2;
    }
    if (pos_out) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double p = b0 * (double)V[3 * i0 + c];
            p = p + b1 * (double)V[3 * i1 + c];
            p = p + b2 * (double)V[3 * i2 + c];
            pos_out[3 * i + c] = (float)p;
        }
    }
}

// ---------------------------------------------------------------------------
// The paper's lattice sampler (Sec. 3.1.1, Sec. 3.1.2): triangle t subdivided
// at resolution r_t holds (r_t + 1)(r_t + 2) / 2 points (Eq. 1) whose
// barycentrics are multiples of 1 / r_t, indexed row by row.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t lattice_points(int64_t r) { return (r + 1) * (r + 2) / 2; }

// Eq. (4): Delta = (8 k) A + 1; r = 1 below Delta = 25, else the positive root
// (sqrt(Delta) - 3) / 2 truncated to a whole resolution.
__device__ __forceinline__ int64_t lattice_resolution(double k, double A)
{
    double delta = 8.0 * k;
    delta = delta * A;
    delta = delta + 1.0;
    if (!(delta >= 25.0)) return 1;
    return (int64_t)floor((sqrt(delta) - 3.0) / 2.0);
}

__global__ void k_lattice_count(const double* __restrict__ area, int64_t T, double k,
                                unsigned long long* __restrict__ cnt)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= T) return;
    cnt[t] = (unsigned long long)lattice_points(lattice_resolution(k, area[t]));
}

// One thread: per-mesh point totals from the inclusive scan of the counts.
__global__ void k_lattice_mesh_counts(const unsigned long long* __restrict__ C, const int64_t* __restrict__ tri_off,
                                      int32_t M, int64_t* __restrict__ counts)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int32_t m = 0; m < M; ++m) {
        const int64_t a = tri_off[m], b = tri_off[m + 1];
        counts[m] = b > a ? (int64_t)(C[b - 1] - (a > 0 ? C[a - 1] : 0ull)) : 0;
    }
}

// Point i of the scene (mesh order, triangle order, then idx in the triangle).
// Eq. (2): row = ceil((sqrt(8 idx + 9) - 3) / 2), corrected with integers to
// f(row - 1) <= idx < f(row); col = idx - f(row - 1).  Eq. (3), completed to a
// partition of unity: w1 = col / r, w2 = (r - row) / r, w3 = (row - col) / r;
// P = (w1 v0 + w2 v1) + w3 v2 in FP64, rounded to FP32; bary = (w2, w3).
__global__ void __launch_bounds__(kBlock)
k_lattice_sample(const float* __restrict__ V, const int32_t* __restrict__ I, const int32_t* __restrict__ tri_mesh,
                 const double* __restrict__ area, const unsigned long long* __restrict__ C, int64_t T, int64_t N,
                 double k, int32_t* __restrict__ tri_out, int32_t* __restrict__ mesh_out,
                 float* __restrict__ bary_out, float* __restrict__ pos_out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    // triangle: the first with inclusive point count above i
    int64_t l = 0, h = T - 1;
    while (l < h) {
        const int64_t mid = l + ((h - l) >> 1);
        if (C[mid] > (unsigned long long)i) h = mid; else l = mid + 1;
    }
    const int64_t t = l;
    const int64_t idx = i - (t > 0 ? (int64_t)C[t - 1] : 0);
    const int64_t r = lattice_resolution(k, area[t]);
    int64_t row = (int64_t)ceil((sqrt(8.0 * (double)idx + 9.0) - 3.0) / 2.0);
    if (row < 0) row = 0;
    while (lattice_points(row) <= idx) ++row;
    while (row > 0 && lattice_points(row - 1) > idx) --row;
    const int64_t col = idx - (row > 0 ? lattice_points(row - 1) : 0);
    const double w1 = (double)col / (double)r;
    const double w2 = (double)(r - row) / (double)r;
    const double w3 = (double)(row - col) / (double)r;
    const int32_t i0 = I[3 * t], i1 = I[3 * t + 1], i2 = I[3 * t + 2];
    if (tri_out) tri_out[i] = (int32_t)t;
    if (mesh_out) mesh_out[i] = tri_mesh[t];
    if (bary_out) {
        bary_out[2 * i] = (float)w2;
        bary_out[2 * i + 1] = (float)w3;
    }
    if (pos_out) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double p = w1 * (double)V[3 * i0 + c];
            p = p + w2 * (double)V[3 * i1 + c];
            p = p + w3 * (double)V[3 * i2 + c];
            pos_out[3 * i + c] = (float)p;
        }
    }
}

// FP64 square root as the sampler evaluates it (same translation unit and flags): the
// canonical area and the square-root warp both need it correctly rounded.
__global__ void k_sqrt_f64(const double* __restrict__ x, double* __restrict__ y, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        y[i] = sqrt(x[i]);
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

void launch_sqrt_f64(const double* x, double* y, int64_t n, hipStream_t s)
{
    if (n > 0) k_sqrt_f64<<<(unsigned)std::min<int64_t>(grid_for(n), 8192), kBlock, 0, s>>>(x, y, n);
}

void launch_tri_area(const float* V, const int32_t* I, const int32_t* tri_mesh, int64_t T, double* area,
                     unsigned long long* max_bits, hipStream_t s)
{
    if (T > 0) k_tri_area<<<grid_for(T), kBlock, 0, s>>>(V, I, tri_mesh, T, area, max_bits);
}

void launch_mesh_scale(const unsigned long long* max_bits, const int64_t* tri_off, int32_t M, int32_t* S,
                       hipStream_t s)
{
    k_mesh_scale<<<grid_for(M), kBlock, 0, s>>>(max_bits, tri_off, M, S);
}

void launch_tri_weight(const double* area, const int32_t* tri_mesh, const int32_t* S, int64_t T,
                       unsigned long long* W, hipStream_t s)
{
    if (T > 0) k_tri_weight<<<grid_for(T), kBlock, 0, s>>>(area, tri_mesh, S, T, W);
}

void launch_mesh_counts(const unsigned long long* C, const int64_t* tri_off, const int32_t* S, int32_t M,
                        double k, int64_t* counts, int64_t* offsets, unsigned long long* mesh_total,
                        hipStream_t s)
{
    k_mesh_counts<<<1, 1, 0, s>>>(C, tri_off, S, M, k, counts, offsets, mesh_total);
}

void launch_sample(const float* V, const int32_t* I, const unsigned long long* C, const int64_t* tri_off,
                   const int64_t* offsets, const unsigned long long* mesh_total, const int32_t* guide,
                   const int64_t* goff, const int32_t* gsh, int32_t M, int64_t N, uint64_t seed, int32_t* tri,
                   int32_t* mesh, float* bary, float* pos, hipStream_t s)
{
    if (N > 0)
        k_sample<<<grid_for(N), kBlock, 0, s>>>(V, I, C, tri_off, offsets, mesh_total, guide, goff, gsh, M, N,
                                                (uint32_t)seed, (uint32_t)(seed >> 32), tri, mesh, bary, pos);
}

void launch_sample_guide(const unsigned long long* C, const int64_t* tri_off, const int64_t* goff,
                         const int32_t* gsh, int32_t M, int64_t G, int32_t* guide, hipStream_t s)
{
    if (G > 0) k_sample_guide<<<grid_for(G), kBlock, 0, s>>>(C, tri_off, goff, gsh, M, G, guide);
}

void launch_lattice_count(const double* area, int64_t T, double k, unsigned long long* cnt, hipStream_t s)
{
    if (T > 0) k_lattice_count<<<grid_for(T), kBlock, 0, s>>>(area, T, k, cnt);
}

void launch_lattice_mesh_counts(const unsigned long long* C, const int64_t* tri_off, int32_t M, int64_t* counts,
                                hipStream_t s)
{
    k_lattice_mesh_counts<<<1, 1, 0, s>>>(C, tri_off, M, counts);
}

void launch_lattice_sample(const float* V, const int32_t* I, const int32_t* tri_mesh, const double* area,
                           const unsigned long long* C, int64_t T, int64_t N, double k, int32_t* tri, int32_t* mesh,
                           float* bary, float* pos, hipStream_t s)
{
    if (N > 0 && T > 0)
        k_lattice_sample<<<grid_for(N), kBlock, 0, s>>>(V, I, tri_mesh, area, C, T, N, k, tri, mesh, bary, pos);
}

}  // namespace gm
