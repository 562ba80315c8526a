// k_field.hip -- neural density field on gfx950 matrix cores.
//
// x -> 96 Fourier features [sin, cos](2 pi f_b x~_a) (f_b = 2^(0.6 b), b = 0..15) ->
// 4 x (64, ReLU) -> 1 -> softplus, trained by mean squared error on the
// normalised densities the method produces.  Every layer product is a chain of
// v_mfma_f32_32x32x16_bf16 (bf16 operands, fp32 accumulation) per wave of 32
// points, in the transposed form Z^T = W^T H^T: weights are the A operand (read
// from LDS), activations the B operand (registers).  The accumulator layout of
// one product (lane = point, rows 8q + 4h + r) is exactly the B-operand layout
// of the next one once the input features of each 16-wide k-step are visited
// in the slot order of slot_feature(); the packed weight image stores every
// matrix in that order, so activations never leave registers between layers.
// The backward pass reuses the same trick for dH = W dZ and takes the weight
// gradients dW = H dZ^T as MFMA products over the 32 points of the wave (a
// transpose of H and dZ through per-wave LDS tiles).  Each wave adds its tiles'
// gradients, in its own tile order, into a slot of its own (plain loads and stores,
// no atomics), and a second kernel sums the slots in slot order: the gradient, and
// so training, is the same bit for bit on every run.  Adam (Kingma and Ba 2015)
// keeps fp32 master weights and moments.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gm_internal.h"
#include "gm_philox.h"

namespace gm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef short i16x8 __attribute__((ext_vector_type(8)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kW = kFieldWidth;              // 64
constexpr int kS1 = 104;                     // LDS row stride (bf16) of the layer-1 weights, padded
constexpr int kSH = 72;                      // LDS row stride (bf16) of a 64-wide weight matrix, padded
constexpr int kOffF1 = 0;                    // forward operand of layer 1: [64 out][104]
constexpr int kMatH = kW * kSH * 2;          // bytes of one 64 x 64 operand
constexpr int kOffF2 = kOffF1 + kW * kS1 * 2;  // forward operands of layers 2..4: [64 out][72]
constexpr int kOffBias = kOffF2 + 3 * kMatH;   // fp32 b1..b4
constexpr int kOffW5 = kOffBias + 4 * kW * 4;  // fp32 w5
constexpr int kOffB5 = kOffW5 + kW * 4;        // fp32 b5 (+ padding)
constexpr int kInfer = kOffB5 + 16;
constexpr int kOffB2 = kInfer;                 // backward operands of layers 2..4: [64 in][72]
constexpr int kPack = kOffB2 + 3 * kMatH;
static_assert(kInfer % 16 == 0 && kPack % 16 == 0, "16-byte copies");

constexpr int kThreads = 256;
constexpr int kTileStride = 40;              // LDS row stride (bf16) of the per-wave 32-point tiles

// slot s of a 16-wide k-step -> feature offset inside the step (the accumulator
// rows 8q + 4h + r of one product, read as the operand of the next)
__host__ __device__ constexpr int slot_feature(int s)
{
    return (s & 7) < 4 ? 4 * (s >> 3) + (s & 7) : 8 + 4 * (s >> 3) + (s & 7) - 4;
}

// layer-1 input slot c = 16 ks + 8 h + j -> feature index 6 band + 2 axis + (sin 0 | cos 1)
__host__ __device__ constexpr int input_feature(int c)
{
    return 6 * ((8 * (c / 16) + c % 8) / 3) + 2 * ((8 * (c / 16) + c % 8) % 3) + (c % 16) / 8;
}

__device__ __forceinline__ f32x16 mfma(const bf16x8& a, const bf16x8& b, const f32x16& c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 lds8(const unsigned char* base, int elem)
{
    return *reinterpret_cast<const bf16x8*>(base + 2 * elem);
}

struct Acts {
    bf16x8 x0[6];     // features, k-steps of layer 1
    bf16x8 h[4][4];   // hidden layers 1..4, k-steps of the next product
};

// log(1 + e) with e = exp(-|o|) in (0, 1], through the hardware exp2/log2: 1 + e rounds away
// at most 2^-24 of the sum, an absolute error below 1e-7 in the output
__device__ __forceinline__ float softplus(float o) { return fmaxf(o, 0.0f) + __logf(1.0f + __expf(-fabsf(o))); }

// The accumulators of a layer start from its bias (in the accumulator layout), so the
// products add onto it.
__device__ __forceinline__ void bias_init(const unsigned char* lds, int layer, int h, f32x16& a0, f32x16& a1)
{
    const float* bias = reinterpret_cast<const float*>(lds + kOffBias) + layer * kW;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int f = 8 * (v >> 2) + 4 * h + (v & 3);
        a0[v] = bias[f];
        a1[v] = bias[32 + f];
    }
}

// ReLU and BF16 rounding of a layer's accumulators into the next product's operand layout.
// The ReLU acts on the rounded values (the same bits as rounding after it: rounding keeps
// the sign), two at a time as 16-bit integers: a BF16 value is negative exactly when its
// sign bit is set, so max(bits, 0) zeroes the negative ones.
__device__ __forceinline__ bf16x8 relu_bf16x8(const f32x16& a, int v0)
{
    const f32x8 f = {a[v0], a[v0 + 1], a[v0 + 2], a[v0 + 3], a[v0 + 4], a[v0 + 5], a[v0 + 6], a[v0 + 7]};
    // the empty asm keeps the conversion and the max apart: combined, the compiler would
    // convert one value per instruction and repack the halves
    u32x4 u = __builtin_bit_cast(u32x4, __builtin_convertvector(f, bf16x8));
    asm("" : "+v"(u));
    return __builtin_bit_cast(bf16x8, __builtin_elementwise_max(__builtin_bit_cast(i16x8, u), i16x8{}));
}

__device__ __forceinline__ void relu_bf16(const f32x16& a0, const f32x16& a1, bf16x8 (&out)[4])
{
    out[0] = relu_bf16x8(a0, 0);
    out[1] = relu_bf16x8(a0, 8);
    out[2] = relu_bf16x8(a1, 0);
    out[3] = relu_bf16x8(a1, 8);
}

// Forward pass of the 32 points of a wave (lane & 31 = point, lane >> 5 = half).
// Returns the pre-softplus output o (same value in both halves).
__device__ __forceinline__ float field_forward(const unsigned char* lds, const FieldGeom& g, float x, float y,
                                               float z, int lane, Acts& A)
{
    const int n = lane & 31, h = lane >> 5;
    const float xt[3] = {(x - g.lo[0]) * g.inv_ext, (y - g.lo[1]) * g.inv_ext, (z - g.lo[2]) * g.inv_ext};
    // slot j of k-step ks: sin/cos pair p = 8 ks + j (band p / 3, axis p % 3); the lane
    // half picks sin (h = 0) or cos (h = 1), taken as sin of the phase + 1/4 revolution
    const float quarter = h ? 0.25f : 0.0f;
#pragma unroll
    for (int ks = 0; ks < 6; ++ks) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int pr = 8 * ks + j;
            // revolutions, reduced to [0, 1) (the hardware sine takes a bounded range)
            const float rev = __builtin_amdgcn_fractf(__builtin_fmaf(g.freq[pr / 3], xt[pr % 3], quarter));
            A.x0[ks][j] = (__bf16)__builtin_amdgcn_sinf(rev);  // sin(2 pi rev)
        }
    }
    f32x16 c0, c1;
    bias_init(lds, 0, h, c0, c1);
#pragma unroll
    for (int ks = 0; ks < 6; ++ks) {
        c0 = mfma(lds8(lds + kOffF1, n * kS1 + 16 * ks + 8 * h), A.x0[ks], c0);
        c1 = mfma(lds8(lds + kOffF1, (32 + n) * kS1 + 16 * ks + 8 * h), A.x0[ks], c1);
    }
    relu_bf16(c0, c1, A.h[0]);
#pragma unroll
    for (int L = 1; L < 4; ++L) {
        const unsigned char* F = lds + kOffF2 + (L - 1) * kMatH;
        f32x16 d0, d1;
        bias_init(lds, L, h, d0, d1);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            d0 = mfma(lds8(F, n * kSH + 16 * ks + 8 * h), A.h[L - 1][ks], d0);
            d1 = mfma(lds8(F, (32 + n) * kSH + 16 * ks + 8 * h), A.h[L - 1][ks], d1);
        }
        relu_bf16(d0, d1, A.h[L]);
    }
    const float* w5 = reinterpret_cast<const float*>(lds + kOffW5);
    float part = 0.0f;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int j = 0; j < 8; ++j) part = __builtin_fmaf(w5[16 * ks + slot_feature(8 * h + j)], (float)A.h[3][ks][j], part);
    return part + __shfl_xor(part, 32, 64) + *reinterpret_cast<const float*>(lds + kOffB5);
}

__device__ __forceinline__ void stage(unsigned char* dst, const unsigned char* __restrict__ src, int bytes)
{
    for (int o = threadIdx.x * 16; o < bytes; o += kThreads * 16)
        *reinterpret_cast<uint4*>(dst + o) = *reinterpret_cast<const uint4*>(src + o);
}

// ---------------------------------------------------------------------------
__global__ void k_field_pack(const float* __restrict__ p, unsigned char* __restrict__ blob, int64_t pack_stride)
{
    const int t = blockIdx.x * kThreads + threadIdx.x;
    p += (int64_t)blockIdx.y * kFieldParams;  // network blockIdx.y
    blob += (int64_t)blockIdx.y * pack_stride;
    __bf16* bf = reinterpret_cast<__bf16*>(blob);
    float* f32 = reinterpret_cast<float*>(blob);
    const int nF1 = kW * kS1, nH = kW * kSH;
    if (t < nF1) {  // layer 1: row = output, column = input slot
        const int i = t / kS1, c = t % kS1;
        bf[t] = (__bf16)(c < kFieldFeat ? p[kFieldOffW[1] + input_feature(c) * kW + i] : 0.0f);
        return;
    }
    int u = t - nF1;
    if (u < 3 * nH) {  // layers 2..4, forward: row = output, column slot -> input feature
        const int L = 2 + u / nH, r = u % nH, i = r / kSH, c = r % kSH;
        float v = 0.0f;
        if (c < kW) v = p[kFieldOffW[L] + (16 * (c / 16) + slot_feature(c % 16)) * kW + i];
        bf[kOffF2 / 2 + u] = (__bf16)v;
        return;
    }
    u -= 3 * nH;
    if (u < 3 * nH) {  // layers 2..4, backward: row = input, column slot -> output feature
        const int L = 2 + u / nH, r = u % nH, k = r / kSH, c = r % kSH;
        float v = 0.0f;
        if (c < kW) v = p[kFieldOffW[L] + k * kW + 16 * (c / 16) + slot_feature(c % 16)];
        bf[kOffB2 / 2 + u] = (__bf16)v;
        return;
    }
    u -= 3 * nH;
    if (u < 4 * kW) {
        f32[kOffBias / 4 + u] = p[kFieldOffB[1 + u / kW] + u % kW];
        return;
    }
    u -= 4 * kW;
    if (u < kW) {
        f32[kOffW5 / 4 + u] = p[kFieldOffW5 + u];
        return;
    }
    u -= kW;
    if (u < 4) f32[kOffB5 / 4 + u] = u == 0 ? p[kFieldOffB5] : 0.0f;
}
constexpr int kPackThreads = kW * kS1 + 6 * kW * kSH + 5 * kW + 4;

__global__ void __launch_bounds__(kThreads) k_field_infer(const unsigned char* __restrict__ blob, FieldGeom g,
                                                          const float* __restrict__ pos, int64_t q,
                                                          float* __restrict__ out, FieldRoute route)
{
    __shared__ __attribute__((aligned(16))) unsigned char s_blob[kInfer];
    stage(s_blob, blob, kInfer);
    __syncthreads();
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    const int64_t tiles = (q + 31) / 32;
    for (int64_t tile = (int64_t)blockIdx.x * (kThreads / 64) + wave; tile < tiles;
         tile += (int64_t)gridDim.x * (kThreads / 64)) {
        // keep the weights in LDS: without this the loop-invariant operand reads are
        // hoisted out of the tile loop and pin the whole weight set in registers
        asm volatile("" ::: "memory");
        const int64_t i = tile * 32 + (lane & 31);
        const bool ok = i < q;
        const int64_t ii = ok ? i : 0;
        Acts A;
        const float o = field_forward(s_blob, g, pos[3 * ii], pos[3 * ii + 1], pos[3 * ii + 2], lane, A);
        if (ok && lane < 32) {
            bool mine = route.m < 0;
            if (!mine) {
                int pm = -1;
                if (route.mesh) {
                    pm = route.mesh[i];
                } else if (route.tri) {
                    const int t = route.tri[i];
                    pm = t >= 0 && t < route.T ? route.tri_mesh[t] : -1;
                }
                mine = pm == route.m;
            }
            if (mine) out[i] = softplus(o);
        }
    }
}

// Routed inference: the points of every network are listed together, one segment per
// mesh in mesh order, each padded to a whole number of kGroup points, segment m starting
// at base[m] (route layout: base [M + 1], then start [M], then count [M]).  A mesh whose
// points already lie contiguously in the input (start[m] >= 0: they are
// start[m] .. start[m] + count[m] - 1, as for samples generated mesh by mesh) is read in
// place; the others through the index list ridx.  Every network evaluates only its own
// mesh's points, all networks in one launch.  A workgroup takes groups of kGroup points
// (one 32-point tile per wave) and stages the weights of the group's network, again only
// when the network changes (its groups run in mesh order).
constexpr int kGroup = 32 * (kThreads / 64);

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) p[i] = v;
}

__device__ __forceinline__ int group_mesh(const int64_t* __restrict__ base, int32_t M, int64_t first)
{
    int lo = 0, hi = M - 1;  // last m with base[m] <= first
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= first) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(kThreads) k_field_infer_routed(const unsigned char* __restrict__ blobs,
                                                                 int64_t pack_stride,
                                                                 const FieldGeom* __restrict__ geoms,
                                                                 const float* __restrict__ pos,
                                                                 const int32_t* __restrict__ ridx,
                                                                 const int64_t* __restrict__ base, int32_t M,
                                                                 float* __restrict__ out)
{
    __shared__ __attribute__((aligned(16))) unsigned char s_blob[kInfer];
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    const int64_t groups = base[M] / kGroup;
    const int64_t* start = base + M + 1;
    const int64_t* count = base + 2 * M + 1;
    int staged = -1;
    FieldGeom g;
    // a contiguous run of groups per workgroup: it crosses at most a few mesh boundaries,
    // so the weights are staged about once per workgroup
    const int64_t g0 = groups * blockIdx.x / gridDim.x, g1 = groups * (blockIdx.x + 1) / gridDim.x;
    for (int64_t gi = g0; gi < g1; ++gi) {
        const int m = group_mesh(base, M, gi * kGroup);
        if (m != staged) {
            __syncthreads();
            stage(s_blob, blobs + (int64_t)m * pack_stride, kInfer);
            __syncthreads();
            staged = m;
            g = geoms[m];
        }
        asm volatile("" ::: "memory");  // weights stay in LDS (see k_field_infer)
        const int64_t slot = gi * kGroup + 32 * wave + (lane & 31);
        const int64_t off = slot - base[m];
        const int64_t s0 = start[m];
        const int64_t i = off >= count[m] ? -1 : s0 >= 0 ? s0 + off : (int64_t)ridx[slot];
        const int64_t ii = i >= 0 ? i : 0;
        Acts A;
        const float o = field_forward(s_blob, g, pos[3 * ii], pos[3 * ii + 1], pos[3 * ii + 2], lane, A);
        if (i >= 0 && lane < 32) out[i] = softplus(o);
    }
}

// point counts of the routed meshes: the point's mesh (mesh[i], or tri_mesh[tri[i]]), when
// it has a network and take[m] is set (NULL: every mesh)
__device__ __forceinline__ int route_mesh(const int32_t* __restrict__ mesh, const int32_t* __restrict__ tri,
                                          const int32_t* __restrict__ tri_mesh, int64_t T,
                                          const uint8_t* __restrict__ take, int32_t M, int64_t i)
{
    int m = -1;
    if (mesh) {
        m = mesh[i];
    } else if (tri) {
        const int t = tri[i];
        m = t >= 0 && t < T ? tri_mesh[t] : -1;
    }
    if (m < 0 || m >= M || (take && !take[m])) return -1;
    return m;
}

// Lanes of a wave that route to the same mesh take their slots with one atomic: the
// wave serves one mesh per round (the first pending lane's), so a wave of points of one
// mesh costs one atomic however many points share it.  Returns this lane's slot among
// the points of its mesh, counted from the value the atomic returned.
// With lo/hi set, the same round also keeps the smallest and largest point index of each
// mesh (lanes hold increasing indices i, so the first and last lane of a round have them).
__device__ __forceinline__ unsigned int wave_reserve(int m, unsigned int* __restrict__ ctr,
                                                     unsigned int* __restrict__ lo = nullptr,
                                                     unsigned int* __restrict__ hi = nullptr, int64_t i = 0)
{
    const int lane = __lane_id();
    uint64_t pending = __ballot(m >= 0);
    unsigned int mine = 0u;
    while (pending) {
        const int lead = __builtin_ctzll(pending);
        const int mm = __builtin_amdgcn_readlane(m, lead);
        const uint64_t same = __ballot(m == mm) & pending;
        if (lo) {
            if (lane == lead) atomicMin(&lo[mm], (unsigned int)i);
            if (lane == 63 - __builtin_clzll(same)) atomicMax(&hi[mm], (unsigned int)i);
        }
        unsigned int base = 0u;
        if (lane == lead) base = atomicAdd(&ctr[mm], (unsigned int)__popcll(same));
        base = __builtin_amdgcn_readlane(base, lead);
        if ((same >> lane) & 1ull) mine = base + (unsigned int)__popcll(same & ((1ull << lane) - 1ull));
        pending &= ~same;
    }
    return mine;
}

// Routing works on chunks of kRouteChunk points per workgroup: the chunk's per-mesh
// counts are gathered in LDS (one LDS atomic per wave and mesh) and added to the global
// ones with one atomic per mesh, so a few hundred global atomics route millions of points.
constexpr int kRouteChunk = 8 * kThreads;
constexpr int kRouteLds = 1024;  // meshes counted in LDS (more: one global atomic per wave and mesh)

__global__ void __launch_bounds__(kThreads) k_route_count(const int32_t* __restrict__ mesh,
                                                          const int32_t* __restrict__ tri,
                                                          const int32_t* __restrict__ tri_mesh, int64_t T,
                                                          const uint8_t* __restrict__ take, int32_t M, int64_t q,
                                                          unsigned int* __restrict__ cnt, unsigned int* __restrict__ part)
{
    // cnt: counts [M], then the smallest [M] and the largest [M] point index per mesh.  With
    // part set, the chunk stores its own three rows at part[chunk][3 M] instead (no two
    // chunks touch one address; k_route_reduce combines them)
    __shared__ unsigned int lc[3 * kRouteLds];
    const bool lds = M <= kRouteLds;
    unsigned int* c = lds ? lc : cnt;
    const int stride = lds ? kRouteLds : M;
    for (int m = threadIdx.x; lds && m < M; m += kThreads) {
        lc[m] = 0u;
        lc[kRouteLds + m] = 0xffffffffu;
        lc[2 * kRouteLds + m] = 0u;
    }
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * kRouteChunk;
    constexpr int kPer = kRouteChunk / kThreads;
    int mm[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {  // every load in flight before the first reservation
        const int64_t i = c0 + j * kThreads + threadIdx.x;
        mm[j] = i < q ? route_mesh(mesh, tri, tri_mesh, T, take, M, i) : -1;
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j)
        (void)wave_reserve(mm[j], c, c + stride, c + 2 * stride, c0 + j * kThreads + threadIdx.x);
    __syncthreads();
    if (lds && part) {
        unsigned int* row = part + (int64_t)blockIdx.x * 3 * M;
        for (int m = threadIdx.x; m < M; m += kThreads) {
            row[m] = lc[m];
            row[M + m] = lc[kRouteLds + m];
            row[2 * M + m] = lc[2 * kRouteLds + m];
        }
        return;
    }
    for (int m = threadIdx.x; lds && m < M; m += kThreads)
        if (lc[m]) {
            atomicAdd(&cnt[m], lc[m]);
            atomicMin(&cnt[M + m], lc[kRouteLds + m]);
            atomicMax(&cnt[2 * M + m], lc[2 * kRouteLds + m]);
        }
}

__global__ void k_route_init(unsigned int* __restrict__ cnt, int32_t M)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < 3 * M) cnt[i] = i >= M && i < 2 * M ? 0xffffffffu : 0u;
}

// one workgroup per mesh: its count, smallest and largest index over the chunks' rows
__global__ void __launch_bounds__(kThreads) k_route_reduce(const unsigned int* __restrict__ part, int64_t chunks,
                                                           int32_t M, unsigned int* __restrict__ cnt)
{
    __shared__ unsigned int rs[kThreads], rl[kThreads], rh[kThreads];
    const int m = blockIdx.x;
    unsigned int s = 0u, lo = 0xffffffffu, hi = 0u;
    for (int64_t c = threadIdx.x; c < chunks; c += kThreads) {
        const unsigned int* row = part + c * 3 * M;
        s += row[m];
        lo = min(lo, row[M + m]);
        hi = max(hi, row[2 * M + m]);
    }
    rs[threadIdx.x] = s; rl[threadIdx.x] = lo; rh[threadIdx.x] = hi;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            rs[threadIdx.x] += rs[threadIdx.x + h];
            rl[threadIdx.x] = min(rl[threadIdx.x], rl[threadIdx.x + h]);
            rh[threadIdx.x] = max(rh[threadIdx.x], rh[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cnt[m] = rs[0];
        cnt[M + m] = rl[0];
        cnt[2 * M + m] = rh[0];
    }
}

// one thread: padded segment starts, the in-place start of every mesh whose points are
// contiguous in the input (largest - smallest index + 1 == count; else -1), the counts,
// and the per-mesh cursors cleared
__global__ void k_route_base(unsigned int* __restrict__ cnt, int32_t M, int64_t* __restrict__ base)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t run = 0;
    for (int m = 0; m < M; ++m) {
        const int64_t c = cnt[m];
        base[m] = run;
        run += (c + kGroup - 1) / kGroup * kGroup;
        const bool contiguous = c > 0 && (int64_t)cnt[2 * M + m] - (int64_t)cnt[M + m] + 1 == c;
        base[M + 1 + m] = contiguous ? (int64_t)cnt[M + m] : -1;
        base[2 * M + 1 + m] = c;
        cnt[m] = 0u;
    }
    base[M] = run;
}

__global__ void __launch_bounds__(kThreads) k_route_scatter(const int32_t* __restrict__ mesh,
                                                            const int32_t* __restrict__ tri,
                                                            const int32_t* __restrict__ tri_mesh, int64_t T,
                                                            const uint8_t* __restrict__ take, int32_t M, int64_t q,
                                                            const int64_t* __restrict__ base,
                                                            unsigned int* __restrict__ cur,
                                                            int32_t* __restrict__ ridx)
{
    constexpr int kPer = kRouteChunk / kThreads;
    __shared__ unsigned int lc[kRouteLds];
    const bool lds = M <= kRouteLds;
    for (int m = threadIdx.x; lds && m < M; m += kThreads) lc[m] = 0u;
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * kRouteChunk;
    int mm[kPer];
    unsigned int rank[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t i = c0 + j * kThreads + threadIdx.x;
        mm[j] = i < q ? route_mesh(mesh, tri, tri_mesh, T, take, M, i) : -1;
        if (mm[j] >= 0 && base[M + 1 + mm[j]] >= 0) mm[j] = -1;  // read in place: no list entry
        rank[j] = wave_reserve(mm[j], lds ? lc : cur);  // rank in the chunk (LDS) or the mesh (global)
    }
    __syncthreads();
    // the chunk's range of each mesh: one global atomic per mesh
    for (int m = threadIdx.x; lds && m < M; m += kThreads)
        lc[m] = lc[m] ? atomicAdd(&cur[m], lc[m]) : 0u;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t i = c0 + j * kThreads + threadIdx.x;
        if (mm[j] >= 0) ridx[base[mm[j]] + (lds ? lc[mm[j]] : 0u) + rank[j]] = (int32_t)i;
    }
}

// a wave's gradient slot: its first tile writes, the later ones add (one lane per entry);
// ONE: every wave takes at most one tile, so every write is the first
template <bool ONE>
__device__ __forceinline__ void put(float* p, float v, bool first) { *p = ONE || first ? v : *p + v; }

template <bool ONE>
__global__ void __launch_bounds__(kThreads) k_field_train(const unsigned char* __restrict__ blob, FieldGeom g,
                                                          FieldTrain t, FieldNets nets)
{
    if (nets.off) {
        // network blockIdx.y of several trained in one launch
        const int m = blockIdx.y;
        const int64_t c = nets.cnt[m];
        if (c == 0) return;
        blob += (int64_t)m * nets.pack_stride;
        g = nets.geom[m];
        t.idx += nets.off[m];
        t.n_idx = c;
        t.key0 ^= (uint32_t)m;
        t.gpart += (int64_t)m * t.slots * kFieldParams;
        t.lpart += (int64_t)m * t.slots;
    }
    __shared__ __attribute__((aligned(16))) unsigned char s_blob[kPack];
    __shared__ __attribute__((aligned(16))) __bf16 s_dz[kThreads / 64][kW][kTileStride];
    __shared__ __attribute__((aligned(16))) __bf16 s_h[kThreads / 64][kFieldFeat][kTileStride];
    stage(s_blob, blob, kPack);
    __syncthreads();
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    const int n = lane & 31, h = lane >> 5;
    const float* w5 = reinterpret_cast<const float*>(s_blob + kOffW5);
    const int tiles = (t.batch + 31) / 32;
    for (int tile = blockIdx.x * (kThreads / 64) + wave; tile < tiles; tile += gridDim.x * (kThreads / 64)) {
        asm volatile("" ::: "memory");  // weights stay in LDS (see k_field_infer)
        // this wave's gradient slot (blockIdx.x * waves + wave < t.slots), written by its
        // first tile and added to by the later ones; a fresh copy of the base each tile:
        // otherwise the ~300 lane-dependent addresses below are hoisted out of the loop
        // and spilled
        const int slot = __builtin_amdgcn_readfirstlane(blockIdx.x * (kThreads / 64) + wave);
        const bool first = tile == slot;
        float* grad = t.gpart + (int64_t)slot * kFieldParams;
        asm volatile("" : "+s"(grad));
        const int j = tile * 32 + n;
        const bool ok = j < t.batch;
        int64_t i = ok ? j : 0;
        if (t.idx) {
            uint32_t c0 = (uint32_t)j, c1 = t.step, c2 = 0u, c3 = 4u;
            philox4x32_10(c0, c1, c2, c3, t.key0, t.key1);
            i = t.idx[(int64_t)(((uint64_t)c0 * (uint64_t)t.n_idx) >> 32)];
        }
        Acts A;
        const float o = field_forward(s_blob, g, t.pos[3 * i], t.pos[3 * i + 1], t.pos[3 * i + 2], lane, A);
        const float y = softplus(o);
        const float diff = ok ? y - t.target[i] : 0.0f;
        const float dO = __fdividef(2.0f * diff * t.inv_batch, 1.0f + __expf(-o));  // d loss / d o
        // loss and the output-layer gradients, reduced over the 32 points of the wave
        float se = h == 0 ? diff * diff : 0.0f, sb = h == 0 ? dO : 0.0f;
#pragma unroll
        for (int d = 1; d < 32; d <<= 1) {
            se += __shfl_xor(se, d, 64);
            sb += __shfl_xor(sb, d, 64);
        }
        if (lane == 0) {
            t.lpart[slot] = ONE || first ? (double)se : t.lpart[slot] + (double)se;
            put<ONE>(&grad[kFieldOffB5], sb, first);
        }
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) {
                float gw = (float)A.h[3][ks][jj] * dO;
#pragma unroll
                for (int d = 1; d < 32; d <<= 1) gw += __shfl_xor(gw, d, 64);
                if (n == 0) put<ONE>(&grad[kFieldOffW5 + 16 * ks + slot_feature(8 * h + jj)], gw, first);
            }
        asm volatile("" ::: "memory");
        // dZ of layer 4 in the accumulator layout
        f32x16 dz0, dz1;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int f = 8 * (v >> 2) + 4 * h + (v & 3);
            dz0[v] = (float)A.h[3][v >> 3][v & 7] > 0.0f ? w5[f] * dO : 0.0f;
            dz1[v] = (float)A.h[3][2 + (v >> 3)][v & 7] > 0.0f ? w5[32 + f] * dO : 0.0f;
        }
#pragma unroll
        for (int L = 4; L >= 1; --L) {
            asm volatile("" ::: "memory");  // one layer at a time (bounds register pressure)
            bf16x8 dzb[4];
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                dzb[v >> 3][v & 7] = (__bf16)dz0[v];
                dzb[2 + (v >> 3)][v & 7] = (__bf16)dz1[v];
                const int f = 8 * (v >> 2) + 4 * h + (v & 3);
                s_dz[wave][f][n] = dzb[v >> 3][v & 7];
                s_dz[wave][32 + f][n] = dzb[2 + (v >> 3)][v & 7];
            }
            if (L >= 2) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) s_h[wave][16 * ks + slot_feature(8 * h + jj)][n] = A.h[L - 2][ks][jj];
            } else {
#pragma unroll
                for (int ks = 0; ks < 6; ++ks)
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) s_h[wave][16 * ks + 8 * h + jj][n] = A.x0[ks][jj];
            }
            asm volatile("" ::: "memory");
            // weight gradient dW[k][i] = sum over points of H[k][p] dZ[i][p]
            const int nk = L == 1 ? 3 : 2;
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int nb = 0; nb < 3; ++nb) {
                    if (nb >= nk) break;
                    f32x16 c = {};
#pragma unroll
                    for (int kp = 0; kp < 2; ++kp) {
                        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&s_dz[wave][mb * 32 + n][16 * kp + 8 * h]);
                        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&s_h[wave][nb * 32 + n][16 * kp + 8 * h]);
                        c = mfma(a, b, c);
                    }
                    const int krow = L == 1 ? input_feature(nb * 32 + n) : nb * 32 + n;
                    float* gW = grad + kFieldOffW[L] + krow * kW + mb * 32 + 4 * h;
#pragma unroll
                    for (int v = 0; v < 16; ++v) put<ONE>(gW + 8 * (v >> 2) + (v & 3), c[v], first);
                }
            // bias gradient: row sums of dZ (lane = output feature)
            {
                float sbias = 0.0f;
#pragma unroll
                for (int p = 0; p < 32; ++p) sbias += (float)s_dz[wave][lane][p];
                put<ONE>(&grad[kFieldOffB[L] + lane], sbias, first);
            }
            if (L >= 2) {
                const unsigned char* Bm = s_blob + kOffB2 + (L - 2) * kMatH;
                f32x16 e0 = {}, e1 = {};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    e0 = mfma(lds8(Bm, n * kSH + 16 * ks + 8 * h), dzb[ks], e0);
                    e1 = mfma(lds8(Bm, (32 + n) * kSH + 16 * ks + 8 * h), dzb[ks], e1);
                }
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    dz0[v] = (float)A.h[L - 2][v >> 3][v & 7] > 0.0f ? e0[v] : 0.0f;
                    dz1[v] = (float)A.h[L - 2][2 + (v >> 3)][v & 7] > 0.0f ? e1[v] : 0.0f;
                }
            }
        }
    }
}

// grad[net][p] = sum of the first `used` slots of network net; loss[net] likewise
// (networks with no training points: cnt[net] == 0, nothing summed, 0).  A workgroup takes
// kRedParams consecutive parameters of one network (blockIdx.y) and splits the slots into
// kRedGroups contiguous runs, one per thread row; each row sums its run in slot order, then
// one thread per parameter adds the rows in row order.  The order of every addition is fixed
// by (used, slot), so the result is the same on every run.
constexpr int kRedParams = 32;
constexpr int kRedGroups = kThreads / kRedParams;

__global__ void k_field_grad_reduce(const float* __restrict__ gpart, const double* __restrict__ lpart, int32_t used,
                                    int32_t slots, const int64_t* __restrict__ cnt, float* __restrict__ grad,
                                    double* __restrict__ loss)
{
    __shared__ float rows[kRedGroups][kRedParams];
    __shared__ double lrows[kThreads];
    const int net = blockIdx.y;
    const bool live = !cnt || cnt[net] > 0;
    const int n = live ? used : 0;
    const int col = threadIdx.x % kRedParams, row = threadIdx.x / kRedParams;
    const int p = blockIdx.x * kRedParams + col;
    const int per = (n + kRedGroups - 1) / kRedGroups;
    const int w0 = row * per, w1 = min(n, w0 + per);
    float sum = 0.0f;
    if (p < kFieldParams) {
        const float* src = gpart + (int64_t)net * slots * kFieldParams + p;
        int w = w0;
        for (; w + 8 <= w1; w += 8) {  // eight loads in flight, added in slot order
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = src[(int64_t)(w + k) * kFieldParams];
#pragma unroll
            for (int k = 0; k < 8; ++k) sum += v[k];
        }
        for (; w < w1; ++w) sum += src[(int64_t)w * kFieldParams];
    }
    rows[row][col] = sum;
    if (blockIdx.x == 0) {
        // the loss: thread i sums slots i, i + kThreads, ... in order, then a fixed pairwise tree
        double l = 0.0;
        for (int w = threadIdx.x; w < n; w += kThreads) l += lpart[(int64_t)net * slots + w];
        lrows[threadIdx.x] = l;
    }
    __syncthreads();
    if (row == 0 && p < kFieldParams) {
        float s = rows[0][col];
        for (int r = 1; r < kRedGroups; ++r) s += rows[r][col];
        grad[(int64_t)net * kFieldParams + p] = s;
    }
    if (blockIdx.x == 0) {
        for (int h = kThreads / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) lrows[threadIdx.x] += lrows[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) loss[net] = lrows[0];
    }
}

__global__ void k_field_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                             float* __restrict__ grad, int64_t count, float lr, float b1, float b2, float eps,
                             float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= count) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    grad[i] = 0.0f;
}

__global__ void k_field_split(int64_t n, uint32_t key0, uint32_t key1, uint32_t threshold, uint32_t* __restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32), c2 = 0u, c3 = 3u;
    philox4x32_10(c0, c1, c2, c3, key0, key1);
    flag[i] = c0 >= threshold ? 1u : 0u;  // 1 = training, 0 = held out
}

__global__ void k_field_select(const uint32_t* __restrict__ flag, const int32_t* __restrict__ mesh, int32_t m,
                               int64_t n, uint32_t* __restrict__ sel)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) sel[i] = flag[i] && mesh[i] == m ? 1u : 0u;
}

__global__ void k_field_compact(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ offs, int64_t n,
                                int32_t* __restrict__ idx)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n && flag[i]) idx[offs[i]] = (int32_t)i;
}

// Held-out error sums per mesh, in a fixed order: workgroup (chunk, m) adds the squared
// error and squared target of the held-out points of mesh m in its chunk of kL2Chunk points
// (each thread its points in index order, then a fixed pairwise tree) into part[m][chunk];
// k_field_l2_sum adds the chunks of each mesh the same way.  No atomics: the gate decision
// is the same on every run.
constexpr int kL2Chunk = 16 * kThreads;

__device__ __forceinline__ void tree_sum2(double* a, double* b)
{
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            a[threadIdx.x] += a[threadIdx.x + h];
            b[threadIdx.x] += b[threadIdx.x + h];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kThreads) k_field_l2(const float* __restrict__ pred, const float* __restrict__ target,
                                                       const int32_t* __restrict__ mesh,
                                                       const uint32_t* __restrict__ flag, int64_t n, int32_t M,
                                                       double* __restrict__ part)
{
    __shared__ double se[kThreads], st[kThreads];
    const int m = blockIdx.y;
    const int64_t c0 = (int64_t)blockIdx.x * kL2Chunk;
    double e = 0.0, s = 0.0;
#pragma unroll 4
    for (int j = 0; j < kL2Chunk / kThreads; ++j) {
        const int64_t i = c0 + j * kThreads + threadIdx.x;
        if (i < n && !flag[i] && mesh[i] == m) {
            const double d = (double)pred[i] - (double)target[i];
            e += d * d;
            s += (double)target[i] * (double)target[i];
        }
    }
    se[threadIdx.x] = e;
    st[threadIdx.x] = s;
    __syncthreads();
    tree_sum2(se, st);
    if (threadIdx.x == 0) {
        part[2 * ((int64_t)m * gridDim.x + blockIdx.x)] = se[0];
        part[2 * ((int64_t)m * gridDim.x + blockIdx.x) + 1] = st[0];
    }
}

__global__ void __launch_bounds__(kThreads) k_field_l2_sum(const double* __restrict__ part, int64_t chunks,
                                                           double* __restrict__ sums)
{
    __shared__ double se[kThreads], st[kThreads];
    const int m = blockIdx.x;
    double e = 0.0, s = 0.0;
    for (int64_t c = threadIdx.x; c < chunks; c += kThreads) {
        e += part[2 * (m * chunks + c)];
        s += part[2 * (m * chunks + c) + 1];
    }
    se[threadIdx.x] = e;
    st[threadIdx.x] = s;
    __syncthreads();
    tree_sum2(se, st);
    if (threadIdx.x == 0) {
        sums[2 * m] = se[0];
        sums[2 * m + 1] = st[0];
    }
}

__global__ void k_gate_flags(const int32_t* __restrict__ mesh, const int32_t* __restrict__ tri,
                             const int32_t* __restrict__ tri_mesh, int64_t T, const uint8_t* __restrict__ gate,
                             int32_t M, int64_t q, uint32_t* __restrict__ need)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= q) return;
    int m = -1;
    if (mesh) m = mesh[i];
    else if (tri) {
        const int t = tri[i];
        if (t >= 0 && t < T) m = tri_mesh[t];
    }
    need[i] = (gate == nullptr || m < 0 || m >= M || gate[m] == 0) ? 1u : 0u;
}

__global__ void k_gather_points(const float* __restrict__ pos, const int32_t* __restrict__ tri,
                                const int32_t* __restrict__ mesh, const uint32_t* __restrict__ need,
                                const uint32_t* __restrict__ offs, int64_t q, float* __restrict__ gpos,
                                int32_t* __restrict__ gtri, int32_t* __restrict__ gmesh, int32_t* __restrict__ gidx)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= q || !need[i]) return;
    const uint32_t j = offs[i];
    gpos[3 * j] = pos[3 * i];
    gpos[3 * j + 1] = pos[3 * i + 1];
    gpos[3 * j + 2] = pos[3 * i + 2];
    gtri[j] = tri ? tri[i] : -1;
    gmesh[j] = mesh ? mesh[i] : -1;
    gidx[j] = (int32_t)i;
}

__global__ void k_scatter_fallback(const float* __restrict__ rho, const int32_t* __restrict__ gidx, int64_t m,
                                   const float* __restrict__ norm, float* __restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= m) return;
    const float d = *norm;
    out[gidx[j]] = d > 0.0f ? rho[j] / d : 0.0f;
}

__global__ void k_used_flags(const uint32_t* __restrict__ need, int64_t q, uint8_t* __restrict__ used)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < q) used[i] = (uint8_t)need[i];
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

size_t field_pack_bytes() { return kPack; }
size_t field_infer_bytes() { return kInfer; }

void launch_field_pack(const float* master, unsigned char* blob, hipStream_t s)
{
    k_field_pack<<<blocks(kPackThreads), kThreads, 0, s>>>(master, blob, 0);
}

void launch_field_pack_nets(const float* master, unsigned char* blob, int32_t M, hipStream_t s)
{
    if (M > 0) k_field_pack<<<dim3(blocks(kPackThreads), (unsigned)M), kThreads, 0, s>>>(master, blob, kPack);
}

void launch_field_infer(const unsigned char* blob, const FieldGeom& g, const float* pos, int64_t q, float* out,
                        const FieldRoute& route, hipStream_t s)
{
    if (q <= 0) return;
    const int64_t tiles = (q + 31) / 32;
    const unsigned grid = (unsigned)std::min<int64_t>((tiles + 3) / 4, 2048);
    k_field_infer<<<grid, kThreads, 0, s>>>(blob, g, pos, q, out, route);
}

int64_t field_route_slots(int64_t q, int32_t M) { return q + (int64_t)kGroup * M; }

int64_t field_route_part_bytes(int64_t q, int32_t M)
{
    const int64_t chunks = (q + kRouteChunk - 1) / kRouteChunk;
    const int64_t b = chunks * 3 * (int64_t)M * 4;
    return M <= kRouteLds && b <= ((int64_t)64 << 20) ? b : 0;
}

void launch_field_infer_routed(const unsigned char* blobs, int64_t pack_stride, const FieldGeom* geoms,
                               const float* pos, int64_t q, float* out, const FieldRoute& route,
                               const uint8_t* take, int32_t M, unsigned int* cnt, unsigned int* part, int64_t* base,
                               int32_t* ridx, hipStream_t s)
{
    if (q <= 0 || M <= 0) return;
    const int64_t slots = field_route_slots(q, M);
    const unsigned chunks = (unsigned)((q + kRouteChunk - 1) / kRouteChunk);
    if (!part) k_route_init<<<blocks(3 * (int64_t)M), kThreads, 0, s>>>(cnt, M);
    k_route_count<<<chunks, kThreads, 0, s>>>(route.mesh, route.tri, route.tri_mesh, route.T, take, M, q, cnt, part);
    if (part) k_route_reduce<<<(unsigned)M, kThreads, 0, s>>>(part, chunks, M, cnt);
    k_route_base<<<1, 1, 0, s>>>(cnt, M, base);
    k_route_scatter<<<chunks, kThreads, 0, s>>>(route.mesh, route.tri, route.tri_mesh, route.T, take, M, q, base,
                                                   cnt, ridx);
    const unsigned grid = (unsigned)std::min<int64_t>(slots / kGroup + 1, 2048);
    k_field_infer_routed<<<grid, kThreads, 0, s>>>(blobs, pack_stride, geoms, pos, ridx, base, M, out);
}

void launch_field_select(const uint32_t* flag, const int32_t* mesh, int32_t m, int64_t n, uint32_t* sel, hipStream_t s)
{
    if (n > 0) k_field_select<<<blocks(n), kThreads, 0, s>>>(flag, mesh, m, n, sel);
}

int32_t field_train_slots(int32_t batch, int32_t M)
{
    const int tiles = (batch + 31) / 32;
    const int waves = kThreads / 64;
    // at most ~256 MB of slots over all networks, at least one workgroup per network
    const int64_t cap = std::max<int64_t>(1, ((int64_t)256 << 20) / ((int64_t)M * waves * kFieldParams * 4));
    const int64_t grid = std::min<int64_t>(std::min<int64_t>((tiles + waves - 1) / waves, 1024), cap);
    return (int32_t)(std::max<int64_t>(grid, 1) * waves);
}

void launch_field_train(const unsigned char* blob, const FieldGeom& g, FieldTrain t, float* grad, double* loss,
                        hipStream_t s)
{
    if (t.batch <= 0) return;
    const int tiles = (t.batch + 31) / 32;
    t.slots = field_train_slots(t.batch, 1);
    if (tiles <= t.slots)
        k_field_train<true><<<(unsigned)(t.slots / (kThreads / 64)), kThreads, 0, s>>>(blob, g, t, FieldNets{});
    else
        k_field_train<false><<<(unsigned)(t.slots / (kThreads / 64)), kThreads, 0, s>>>(blob, g, t, FieldNets{});
    k_field_grad_reduce<<<dim3((kFieldParams + kRedParams - 1) / kRedParams, 1), kThreads, 0, s>>>(
        t.gpart, t.lpart, std::min(tiles, t.slots), t.slots, nullptr, grad, loss);
}

void launch_field_train_nets(const unsigned char* blob, const FieldNets& nets, int32_t M, FieldTrain t, float* grad,
                             double* loss, hipStream_t s)
{
    if (t.batch <= 0 || M <= 0) return;
    const int tiles = (t.batch + 31) / 32;
    t.slots = field_train_slots(t.batch, M);
    const dim3 grid((unsigned)(t.slots / (kThreads / 64)), (unsigned)M);
    if (tiles <= t.slots)
        k_field_train<true><<<grid, kThreads, 0, s>>>(blob, FieldGeom{}, t, nets);
    else
        k_field_train<false><<<grid, kThreads, 0, s>>>(blob, FieldGeom{}, t, nets);
    k_field_grad_reduce<<<dim3((kFieldParams + kRedParams - 1) / kRedParams, (unsigned)M), kThreads, 0, s>>>(
        t.gpart, t.lpart, std::min(tiles, t.slots), t.slots, nets.cnt, grad, loss);
}

void launch_field_adam(float* master, float* m, float* v, float* grad, int64_t count, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s)
{
    if (count > 0)
        k_field_adam<<<blocks(count), kThreads, 0, s>>>(master, m, v, grad, count, lr, b1, b2, eps, c1, c2);
}

void launch_field_split(int64_t n, uint32_t key0, uint32_t key1, uint32_t threshold, uint32_t* flag, hipStream_t s)
{
    if (n > 0) k_field_split<<<blocks(n), kThreads, 0, s>>>(n, key0, key1, threshold, flag);
}

void launch_field_compact(const uint32_t* flag, const uint32_t* offs, int64_t n, int32_t* idx, hipStream_t s)
{
    if (n > 0) k_field_compact<<<blocks(n), kThreads, 0, s>>>(flag, offs, n, idx);
}

int64_t field_l2_part_bytes(int64_t n, int32_t M) { return 16 * ((n + kL2Chunk - 1) / kL2Chunk) * (int64_t)M; }

void launch_field_l2(const float* pred, const float* target, const int32_t* mesh, const uint32_t* flag, int64_t n,
                     int32_t M, double* part, double* sums, hipStream_t s)
{
    if (M <= 0) return;
    const int64_t chunks = (n + kL2Chunk - 1) / kL2Chunk;
    if (chunks > 0)
        k_field_l2<<<dim3((unsigned)chunks, (unsigned)M), kThreads, 0, s>>>(pred, target, mesh, flag, n, M, part);
    k_field_l2_sum<<<(unsigned)M, kThreads, 0, s>>>(part, chunks, sums);
}

void launch_gate_flags(const int32_t* mesh, const int32_t* tri, const int32_t* tri_mesh, int64_t T,
                       const uint8_t* gate, int32_t M, int64_t q, uint32_t* need, hipStream_t s)
{
    if (q > 0) k_gate_flags<<<blocks(q), kThreads, 0, s>>>(mesh, tri, tri_mesh, T, gate, M, q, need);
}

void launch_gather_points(const float* pos, const int32_t* tri, const int32_t* mesh, const uint32_t* need,
                          const uint32_t* offs, int64_t q, float* gpos, int32_t* gtri, int32_t* gmesh, int32_t* gidx,
                          hipStream_t s)
{
    if (q > 0) k_gather_points<<<blocks(q), kThreads, 0, s>>>(pos, tri, mesh, need, offs, q, gpos, gtri, gmesh, gidx);
}

void launch_scatter_fallback(const float* rho, const int32_t* gidx, int64_t m, const float* norm, float* out,
                             hipStream_t s)
{
    if (m > 0) k_scatter_fallback<<<blocks(m), kThreads, 0, s>>>(rho, gidx, m, norm, out);
}

void launch_used_flags(const uint32_t* need, int64_t q, uint8_t* used, hipStream_t s)
{
    if (q > 0) k_used_flags<<<blocks(q), kThreads, 0, s>>>(need, q, used);
}

}  // namespace gm
