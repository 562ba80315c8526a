// k_density.hip -- fixation density accumulation on surface samples
// (Sec. 3.2.1 angular Gaussian, Sec. 3.2.2 visibility, Sec. 3.2.3 normalisation,
// Sec. 3.3.2 4-sigma truncation), for gfx950.
//
// Work decomposition.  Samples are first put in spatial (Morton) order.  A
// workgroup owns a tile of 256*SPL consecutive samples (SPL per lane, held in
// VGPRs in tile-local coordinates) and one chunk of the fixations.  Fixations
// stream through LDS in blocks of kFB; every lane evaluates the cheap cone gate
// for its SPL samples against each fixation (8 FMA per pair, all FMA):
//     d = r.x' + c0,  m = a.x' + cc - kappa |x'|^2,  s = d|d| + m
// with x' = x - (tile origin), c0 = -r.e', a = 2 kappa e', cc = -kappa |e'|^2,
// kappa = |r|^2 / (1 + 16 sigma^2) slightly widened, so that s > 0 for every
// pair inside the 4-sigma cone (d > 0 and tan(phi) <= 4 sigma).  Only when some
// lane of the wave passes does the wave take the exact path: the pair value in
// compensated FP32 (TwoSum for p = x - e, FMA difference of products for p x r),
// then the visibility of the passing lanes as one packet (all rays share the eye)
// through the BVH, with wave-uniform node and triangle fetches.  Contributions
// are accumulated per lane as exact 64-bit fixed point, so the final value does
// not depend on the order of work.
//
// Built with -ffp-contract=off: every fused multiply-add below is written out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "gm_internal.h"

namespace gm {
namespace {

constexpr int kThreads = 256;
constexpr int kFB = 128;  // fixations per LDS block

// Records whose address is the same for the whole wave are read through the
// constant address space, which lets the compiler use scalar (SMEM) loads.
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(4))) const vf4* CVec4Ptr;

__device__ __forceinline__ BvhNode load_node(const BvhNode* base, int i)
{
    const CVec4Ptr q = (CVec4Ptr)(base + i);
    const vf4 a = q[0], b = q[1], c = q[2], d = q[3];
    BvhNode n;
    n.lo0[0] = a.x; n.lo0[1] = a.y; n.lo0[2] = a.z;
    n.hi0[0] = a.w; n.hi0[1] = b.x; n.hi0[2] = b.y;
    n.lo1[0] = b.z; n.lo1[1] = b.w; n.lo1[2] = c.x;
    n.hi1[0] = c.y; n.hi1[1] = c.z; n.hi1[2] = c.w;
    n.child0 = __float_as_int(d.x); n.child1 = __float_as_int(d.y);
    n.count0 = __float_as_int(d.z); n.count1 = __float_as_int(d.w);
    return n;
}

__device__ __forceinline__ BvhTri load_tri(const BvhTri* base, int i)
{
    const CVec4Ptr q = (CVec4Ptr)(base + i);
    const vf4 a = q[0], b = q[1], c = q[2];
    BvhTri t;
    t.v0[0] = a.x; t.v0[1] = a.y; t.v0[2] = a.z;
    t.v1[0] = a.w; t.v1[1] = b.x; t.v1[2] = b.y;
    t.v2[0] = b.z; t.v2[1] = b.w; t.v2[2] = c.x;
    t.id = __float_as_int(c.y); t.mesh = __float_as_int(c.z); t.pad = 0;
    return t;
}

// the same record at a lane-dependent index (vector loads)
__device__ __forceinline__ BvhTri load_tri_v(const BvhTri* base, int i)
{
    const float4* q = reinterpret_cast<const float4*>(base + i);
    const float4 a = q[0], b = q[1], c = q[2];
    BvhTri t;
    t.v0[0] = a.x; t.v0[1] = a.y; t.v0[2] = a.z;
    t.v1[0] = a.w; t.v1[1] = b.x; t.v1[2] = b.y;
    t.v2[0] = b.z; t.v2[1] = b.w; t.v2[2] = c.x;
    t.id = __float_as_int(c.y); t.mesh = __float_as_int(c.z); t.pad = 0;
    return t;
}

__device__ __forceinline__ FixRec load_fix(const FixRec* base, int i)
{
    const CVec4Ptr q = (CVec4Ptr)(base + i);
    const vf4 a = q[0], b = q[1];
    FixRec f;
    f.ex = a.x; f.ey = a.y; f.ez = a.z; f.rx = a.w;
    f.ry = b.x; f.rz = b.y; f.w = b.z; f.kappa = b.w;
    return f;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// exact pair value
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& err)
{
    s = a + b;
    const float bb = s - a;
    err = (a - (s - bb)) + (b - bb);
}

// a*b - c*d with one rounding error (Kahan's FMA algorithm)
__device__ __forceinline__ float diff_of_products(float a, float b, float c, float d)
{
    const float w = c * d;
    const float e = __builtin_fmaf(-c, d, w);
    const float f = __builtin_fmaf(a, b, -w);
    return f + e;
}

// |p x r|^2 and p.r for p = x - e, with p carried as a TwoSum pair (hi + lo) and the
// cross product's differences of products with one rounding each
__device__ __forceinline__ void pair_terms(float x, float y, float z, float ex, float ey, float ez, float rx,
                                           float ry, float rz, float& q, float& d1)
{
    float phx, plx, phy, ply, phz, plz;
    two_sum(x, -ex, phx, plx);
    two_sum(y, -ey, phy, ply);
    two_sum(z, -ez, phz, plz);
    const float cx = diff_of_products(phy, rz, phz, ry) + (ply * rz - plz * ry);
    const float cy = diff_of_products(phz, rx, phx, rz) + (plz * rx - plx * rz);
    const float cz = diff_of_products(phx, ry, phy, rx) + (plx * ry - ply * rx);
    q = __builtin_fmaf(cx, cx, __builtin_fmaf(cy, cy, cz * cz));
    const float lo = __builtin_fmaf(plx, rx, __builtin_fmaf(ply, ry, plz * rz));
    d1 = __builtin_fmaf(phx, rx, __builtin_fmaf(phy, ry, __builtin_fmaf(phz, rz, lo)));
}

// Returns g (0 outside the 4-sigma cone).  tan^2(phi) = |p x r|^2 / (p.r)^2 with the
// gaze left unnormalised (its length cancels).
__device__ __forceinline__ float pair_value(float x, float y, float z, float ex, float ey, float ez, float rx,
                                            float ry, float rz, float w, float cone2, float kexp)
{
    float q, d1;
    pair_terms(x, y, z, ex, ey, ez, rx, ry, rz, q, d1);
    const float d12 = d1 * d1;
    if (!(d1 > 0.0f) || !(q <= cone2 * d12)) return 0.0f;
    const float t2 = q / d12;
    return w * exp2f(-t2 * kexp);
}

// ---------------------------------------------------------------------------
// packet visibility: every active lane holds one segment between its point and the
// wave's eye
// ---------------------------------------------------------------------------
// A visibility segment starts at the surface point x (t = 0) and ends at the eye e
// (t = 1): t = 1 - tau in the parameter tau of the segment e + tau (x - e), so a
// triangle occludes when it crosses at kEpsV < t < 1.  Starting at the point keeps
// the triangles near it (the ones a segment grazes when the eye sees the point almost
// edge-on) in coordinates of their own small size: vertices relative to the eye carry
// FP32 rounding of ~1e-7 of the eye distance, which the shear amplifies by the inverse
// incidence cosine at grazing incidence.
struct Seg {
    float ix, iy, iz;  // 1 / direction (finite)
    float qx, qy, qz;  // -x / direction
    float sx, sy;      // watertight shear: d[kx] / d[kz], d[ky] / d[kz]
    float tz;          // d[kz]
    int kx, ky, kz;    // axis order of the shear
};

constexpr float kTlo = (float)kEpsV;  // t of the segment's point end at which occluders start

__device__ __forceinline__ float safe_inv(float d)
{
    return fabsf(d) > 1e-30f ? 1.0f / d : copysignf(1e30f, d);
}

__device__ __forceinline__ float pick(int k, float a, float b, float c) { return k == 0 ? a : (k == 1 ? b : c); }

// Dominant axis kz of d and the other two, swapped when d[kz] < 0 so the shear keeps
// the triangle's winding.
__device__ __forceinline__ void axis_order(float dx, float dy, float dz, int& kx, int& ky, int& kz)
{
    const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    kz = ax > ay ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    kx = kz == 2 ? 0 : kz + 1;
    ky = kx == 2 ? 0 : kx + 1;
    if (pick(kz, dx, dy, dz) < 0.0f) {
        const int t = kx;
        kx = ky;
        ky = t;
    }
}

// The other two axes after kz in cyclic order.  The segment test counts both
// windings, so the order need not follow the sign of d[kz].
__device__ __forceinline__ void cyclic_axes(int kz, int& kx, int& ky)
{
    kx = kz == 2 ? 0 : kz + 1;
    ky = kx == 2 ? 0 : kx + 1;
}

__device__ __forceinline__ int dominant_axis(float dx, float dy, float dz)
{
    const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    return ax > ay ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
}

// The shear axis of a visibility segment with direction d under a fixation whose gaze
// has dominant axis gz: gz while d keeps at least 0.4 of its length along it (every
// in-cone segment while the cone half-angle is below ~14 degrees), else d's own
// dominant axis.  A lane's choice depends on its own segment only, so its arithmetic
// does not depend on the other segments of its packet.
__device__ __forceinline__ int segment_axis(int gz, float dx, float dy, float dz)
{
    const float dk = pick(gz, dx, dy, dz);
    return dk * dk >= 0.16f * (dx * dx + dy * dy + dz * dz) ? gz : dominant_axis(dx, dy, dz);
}

// Segment from the point x (t = 0) to the eye e (t = 1), sheared along the given axis
// order; the slab tests of box_hit_signed01 / box_hit01 clamp to [kTlo, 1].
__device__ __forceinline__ Seg make_seg(float xx, float xy, float xz, float ex, float ey, float ez, int kx, int ky,
                                        int kz)
{
    Seg s;
    const float dx = ex - xx, dy = ey - xy, dz = ez - xz;
    s.ix = safe_inv(dx); s.iy = safe_inv(dy); s.iz = safe_inv(dz);
    s.qx = -xx * s.ix; s.qy = -xy * s.iy; s.qz = -xz * s.iz;
    s.kx = kx; s.ky = ky; s.kz = kz;
    const float dkz = pick(kz, dx, dy, dz);
    s.sx = pick(kx, dx, dy, dz) / dkz;
    s.sy = pick(ky, dx, dy, dz) / dkz;
    s.tz = dkz;
    return s;
}

// Slab test when every segment of the packet has the same direction signs: the
// node copy of that octant stores each axis' near plane first, so no per-lane
// min/max is needed.
__device__ __forceinline__ bool box_hit_signed(const Seg& s, const float* near, const float* far, float tmax)
{
    const float nx = __builtin_fmaf(near[0], s.ix, s.qx), fx = __builtin_fmaf(far[0], s.ix, s.qx);
    const float ny = __builtin_fmaf(near[1], s.iy, s.qy), fy = __builtin_fmaf(far[1], s.iy, s.qy);
    const float nz = __builtin_fmaf(near[2], s.iz, s.qz), fz = __builtin_fmaf(far[2], s.iz, s.qz);
    const float tn = fmaxf(fmaxf(nx, ny), fmaxf(nz, 0.0f));
    const float tf = fminf(fminf(fx, fy), fminf(fz, tmax));
    return tn <= tf;
}

__device__ __forceinline__ bool box_hit(const Seg& s, const float* lo, const float* hi, float tmax)
{
    const float t0x = __builtin_fmaf(lo[0], s.ix, s.qx), t1x = __builtin_fmaf(hi[0], s.ix, s.qx);
    const float t0y = __builtin_fmaf(lo[1], s.iy, s.qy), t1y = __builtin_fmaf(hi[1], s.iy, s.qy);
    const float t0z = __builtin_fmaf(lo[2], s.iz, s.qz), t1z = __builtin_fmaf(hi[2], s.iz, s.qz);
    const float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
    const float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
    return tn <= tf;
}

// The slab tests of a segment from make_seg: entry and exit clamped to [kTlo, 1], the
// part of the segment where occluders count (the clamp is a three-input median, one
// instruction each), and a hit when the entry lies strictly below the exit.  The
// strict comparison drops only boxes the segment meets in a single point, and the box
// padding keeps every triangle hit strictly inside.
// The slab parameters are clamped to [0, 1] by the multiply-adds themselves (the clamp bit
// of v_fma_f32, no extra instruction).  With M the largest entry and m the smallest exit
// parameter, the segment part [kTlo, 1] meets the box iff max(M, kTlo) < min(m, 1), which
// for clamped values C is max(C(M), kTlo) < C(m): one max and one compare.
__device__ __forceinline__ float fma01(float a, float b, float c)
{
    return __builtin_amdgcn_fmed3f(__builtin_fmaf(a, b, c), 0.0f, 1.0f);
}

__device__ __forceinline__ bool box_hit_signed01(const Seg& s, const float* near, const float* far)
{
    const float nx = fma01(near[0], s.ix, s.qx), fx = fma01(far[0], s.ix, s.qx);
    const float ny = fma01(near[1], s.iy, s.qy), fy = fma01(far[1], s.iy, s.qy);
    const float nz = fma01(near[2], s.iz, s.qz), fz = fma01(far[2], s.iz, s.qz);
    const float tn = fmaxf(fmaxf(fmaxf(nx, ny), nz), kTlo);
    const float tf = fminf(fminf(fx, fy), fz);
    return tn < tf;
}

__device__ __forceinline__ bool box_hit01(const Seg& s, const float* lo, const float* hi)
{
    const float t0x = fma01(lo[0], s.ix, s.qx), t1x = fma01(hi[0], s.ix, s.qx);
    const float t0y = fma01(lo[1], s.iy, s.qy), t1y = fma01(hi[1], s.iy, s.qy);
    const float t0z = fma01(lo[2], s.iz, s.qz), t1z = fma01(hi[2], s.iz, s.qz);
    const float tn = fmaxf(fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fminf(t0z, t1z)), kTlo);
    const float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z));
    return tn < tf;
}

// Triangle vertices relative to a segment's start (a ray's eye, or a visibility
// segment's point), in the axis order of the record copy the wave reads (the start is
// passed in that same order).
struct TriEye {
    float ax, ay, az, bx, by, bz, cx, cy, cz;
};

__device__ __forceinline__ TriEye tri_eye(const BvhTri& t, float e0, float e1, float e2)
{
    TriEye u;
    u.ax = t.v0[0] - e0; u.ay = t.v0[1] - e1; u.az = t.v0[2] - e2;
    u.bx = t.v1[0] - e0; u.by = t.v1[1] - e1; u.bz = t.v1[2] - e2;
    u.cx = t.v2[0] - e0; u.cy = t.v2[1] - e1; u.cz = t.v2[2] - e2;
    return u;
}

// Watertight segment/triangle test (Woop, Benthin and Wald, JCGT 2013): shear the
// triangle into the segment's frame, three edge functions with inclusive edges,
// FP64 re-evaluation when an edge function is exactly zero; hit when the
// parameter t = T/det lies in (kTlo, 1).  Returns the wave mask of the lanes of
// `amask` (the lanes testing) that hit.  With UNI the vertices are already in
// the segment's axis order; otherwise they are in x, y, z order and each lane
// permutes them.  Both windings count, so the order of kx and ky does not matter.
// Predicates are formed as wave masks of single compares (scalar ANDs) rather than
// as per-lane booleans.
template <bool UNI>
__device__ __forceinline__ uint64_t seg_tri(const Seg& s, const TriEye& u, uint64_t amask)
{
    float akx, aky, akz, bkx, bky, bkz, ckx, cky, ckz;
    if (UNI) {
        akx = u.ax; aky = u.ay; akz = u.az;
        bkx = u.bx; bky = u.by; bkz = u.bz;
        ckx = u.cx; cky = u.cy; ckz = u.cz;
    } else {
        akx = pick(s.kx, u.ax, u.ay, u.az); aky = pick(s.ky, u.ax, u.ay, u.az); akz = pick(s.kz, u.ax, u.ay, u.az);
        bkx = pick(s.kx, u.bx, u.by, u.bz); bky = pick(s.ky, u.bx, u.by, u.bz); bkz = pick(s.kz, u.bx, u.by, u.bz);
        ckx = pick(s.kx, u.cx, u.cy, u.cz); cky = pick(s.ky, u.cx, u.cy, u.cz); ckz = pick(s.kz, u.cx, u.cy, u.cz);
    }
    const float Ax = __builtin_fmaf(-s.sx, akz, akx);
    const float Ay = __builtin_fmaf(-s.sy, akz, aky);
    const float Bx = __builtin_fmaf(-s.sx, bkz, bkx);
    const float By = __builtin_fmaf(-s.sy, bkz, bky);
    const float Cx = __builtin_fmaf(-s.sx, ckz, ckx);
    const float Cy = __builtin_fmaf(-s.sy, ckz, cky);
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    float lo = fminf(fminf(U, V), W), hi = fmaxf(fmaxf(U, V), W);
    const float amin = fminf(fminf(fabsf(U), fabsf(V)), fabsf(W));
    // Most tests miss for every lane: edge functions of both signs and none zero,
    // exactly when (lo * hi) * amin < 0 (an underflow to -0 only sends the wave on
    // to the full test).
    if ((ballot(!((lo * hi) * amin < 0.0f)) & amask) == 0) return 0;
    const uint64_t zero = ballot(amin == 0.0f) & amask;
    if (__builtin_amdgcn_inverse_ballot_w64(zero)) {
        // rare: keep it a real branch (the empty asm stops the compiler from
        // evaluating the FP64 products for every lane and selecting afterwards)
        asm volatile("" ::: "memory");
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
        lo = fminf(fminf(U, V), W);
        hi = fmaxf(fmaxf(U, V), W);
    }
    const float det = U + V + W;
    // t = T' / (det d[kz]) with T' = U akz + V bkz + W ckz: scale T' by the sign of
    // det d[kz] so the range test reads kTlo |d[kz]| |det| < T' < |d[kz]| |det|
    const float Tp = __builtin_fmaf(W, ckz, __builtin_fmaf(V, bkz, U * akz));
    const float Ts = __uint_as_float(__float_as_uint(Tp) ^ ((__float_as_uint(det) ^ __float_as_uint(s.tz)) & 0x80000000u));
    const float lim = fabsf(s.tz) * fabsf(det);
    const uint64_t mixed = ballot(lo < 0.0f) & ballot(hi > 0.0f);
    return amask & ~mixed & ballot(det != 0.0f) & ballot(Ts > kTlo * lim) & ballot(Ts < lim);
}

// Work of packet traversals (wave level): node visits, triangle tests (one per
// triangle tested by at least one lane).
struct TravCount {
    uint32_t nodes = 0, tests = 0;
};

// Packet visibility.  Every lane carries up to R segments (R sample slots of the
// wave), all ending at the wave's eye; `active[r]` marks the segments to test and
// occ[r] receives the answer.  One traversal serves all R * 64 segments: the node
// index is wave-uniform (scalar loads), each lane tests its own segments against both
// child boxes, children are visited eye side first (by the node's split axis and the
// octant `oct` of the eye-to-point directions) and the stack is one VGPR, lane i
// holding entry i.  Per-lane predicates are kept as 64-bit wave masks (scalar
// registers) rather than per-lane booleans.
// `tris` is the record copy whose axis order matches the segments' start points
// `org[r]` (each lane's point, passed in that order): with UNI the packet's shared
// order, otherwise copy 2 (x, y, z) and each lane permutes.  With UNI the packet's
// segments also share their direction signs and `nodes` is the node copy of the
// octant of their (point-to-eye) directions; otherwise the plain copy.
template <int R, bool UNI>
__device__ void occluded_packet(const BvhNode* __restrict__ nodes, const BvhTri* __restrict__ tris,
                                const float (&org)[R][3], int oct, const Seg (&sg)[R],
                                const int (&own_tri)[R], const int (&own_mesh)[R], int mode,
                                const bool (&active)[R], bool (&occ)[R], TravCount& visits)
{
    const int lane = lane_id();
    uint64_t live[R], hit[R];
    uint64_t alive = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        live[r] = ballot(active[r]);
        hit[r] = 0;
        alive |= live[r];
    }
    // self occlusion: only triangles of the segment's own mesh occlude
    const uint64_t self_only = mode == 1 ? ~0ull : 0ull;
    int stack = 0;
    int sp = 0;
    int node = 0;
    while (alive != 0) {
        const BvhNode nd = load_node(nodes, node);
        ++visits.nodes;
        uint64_t h0[R], h1[R];
        uint64_t any0 = 0, any1 = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (UNI) {
                h0[r] = ballot(box_hit_signed01(sg[r], nd.lo0, nd.hi0)) & live[r];
                h1[r] = ballot(box_hit_signed01(sg[r], nd.lo1, nd.hi1)) & live[r];
            } else {
                h0[r] = ballot(box_hit01(sg[r], nd.lo0, nd.hi0)) & live[r];
                h1[r] = ballot(box_hit01(sg[r], nd.lo1, nd.hi1)) & live[r];
            }
            any0 |= h0[r];
            any1 |= h1[r];
        }
        // near child first: child 0 lies lower along the node's split axis, so it is
        // the near one unless the packet runs towards -axis
        const bool swap = (oct >> ((nd.count0 >> kSplitAxisShift) & 3)) & 1;
        int next = -1;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const bool first = (c == 0) != swap;  // c == 0: the near child
            if ((first ? any0 : any1) == 0) continue;
            const int child = first ? nd.child0 : nd.child1;
            const int count = (first ? nd.count0 : nd.count1) & kCountMask;
            if (child < 0) {
                // each record is fetched when its turn comes (fewer scalar registers held
                // across the leaf; see the occupancy note at k_density)
                const BvhTri* leaf = tris + (~child);
                BvhTri tr[kLeafMax];
#pragma unroll
                for (int k = 0; k < kLeafMax; ++k) {
                    if (k >= count) break;
                    tr[k] = load_tri(leaf, k);
                    // both parts of the record (vertices; id and mesh) arrive before the
                    // skip test, one load latency rather than two in sequence
                    asm volatile("" ::"s"(tr[k].v0[0]), "s"(tr[k].id));
                    uint64_t tm[R];
                    uint64_t tany = 0;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        uint64_t skip = ballot(tr[k].id == own_tri[r]);
                        if (self_only != 0) {
                            // a real (uniform) branch: selected with a mask, the compare
                            // would run in full mode too
                            asm volatile("" ::: "memory");
                            skip |= ballot(tr[k].mesh != own_mesh[r]);
                        }
                        tm[r] = (first ? h0[r] : h1[r]) & ~hit[r] & ~skip;
                        tany |= tm[r];
                    }
                    if (tany == 0) continue;
                    ++visits.tests;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        if (tm[r] == 0) continue;
                        hit[r] |= seg_tri<UNI>(sg[r], tri_eye(tr[k], org[r][0], org[r][1], org[r][2]), tm[r]);
                    }
                }
                alive = 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    live[r] &= ~hit[r];
                    alive |= live[r];
                }
                if (alive == 0) break;
            } else if (next < 0) {
                next = child;
            } else {
                stack = lane == sp ? child : stack;  // push
                ++sp;
            }
        }
        if (alive == 0) break;
        if (next < 0) {
            if (sp == 0) break;
            --sp;
            next = __builtin_amdgcn_readlane(stack, sp);  // pop
        }
        node = uniform(next);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) occ[r] = __builtin_amdgcn_inverse_ballot_w64(hit[r]);
}

// ---------------------------------------------------------------------------
// The back-face rule.  A point x on a triangle of a closed mesh M (a surface that bounds
// a solid: winding number 0 outside, +1 across a triangle against its normal), seen from
// an eye e outside M's bounding box with (e - x) . n < 0, has some triangle of M crossing
// the open segment (e, x): the winding number is 0 at e and at least 1 just behind x.  If
// no triangle of M but x's own crosses the segment's last stretch, from x to
// y = x + kEpsV (e - x), the crossing lies between e and y, at tau < 1 - kEpsV in the
// oracle's parameter, and the pair is occluded: no traversal is needed.  That stretch is
// shorter than rmax (the rule is used for segments up to rmax / kEpsV long), so only
// triangles of M within rmax of x can cross it; they are listed per point by the packet
// walk below, and each is tested against the stretch with margins that make the test
// answer "may cross" whenever FP32 rounding could hide a crossing.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float box_dist2(float x, float y, float z, const float* lo, const float* hi)
{
    const float dx = fmaxf(fmaxf(lo[0] - x, x - hi[0]), 0.0f);
    const float dy = fmaxf(fmaxf(lo[1] - y, y - hi[1]), 0.0f);
    const float dz = fmaxf(fmaxf(lo[2] - z, z - hi[2]), 0.0f);
    return __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
}

// The back-face data of one point per lane (points of a wave close together, as the
// sorted points are): the unit normal of its own triangle t scaled by the point's
// distance D to the triangle's edges (in its plane), and the record indices (plain x, y,
// z copy) of the triangles of its mesh m, other than t, whose boxes come within rmax of
// it, by one packet walk of the scene BVH per wave (wave-uniform node, the lane's sphere
// against both child boxes; squared distances against rmax^2 widened by 1e-3).  cnt =
// -1: the rule does not apply (no closed mesh, degenerate triangle, more than kBfCand
// neighbours).  Every lane of the wave must call it.
__device__ __forceinline__ void backface_point(float px, float py, float pz, int t, int m, bool on,
                                               const float* __restrict__ V, const int32_t* __restrict__ I,
                                               const uint8_t* __restrict__ closed,
                                               const BvhNode* __restrict__ nodes, const BvhTri* __restrict__ tris,
                                               float rmax, float& nx, float& ny, float& nz, int& cnt,
                                               int (&cand)[kBfCand])
{
    const int lane = lane_id();
    nx = ny = nz = 0.0f;
    on = on && t >= 0 && m >= 0 && closed[m] != 0;
    if (on) {
        const int i0 = I[3 * t], i1 = I[3 * t + 1], i2 = I[3 * t + 2];
        const float ax = V[3 * i0], ay = V[3 * i0 + 1], az = V[3 * i0 + 2];
        const float ux = V[3 * i1] - ax, uy = V[3 * i1 + 1] - ay, uz = V[3 * i1 + 2] - az;
        const float vx = V[3 * i2] - ax, vy = V[3 * i2 + 1] - ay, vz = V[3 * i2 + 2] - az;
        nx = diff_of_products(uy, vz, uz, vy);
        ny = diff_of_products(uz, vx, ux, vz);
        nz = diff_of_products(ux, vy, uy, vx);
        const float l2 = __builtin_fmaf(nx, nx, __builtin_fmaf(ny, ny, nz * nz));
        on = l2 > 0.0f && isfinite(l2);
        // distance to the edge opposite each vertex: its barycentric times 2 area / edge
        // length (2 area = |n|); a point outside any edge gets 0
        const float wx = px - ax, wy = py - ay, wz = pz - az;
        const float c1x = diff_of_products(wy, vz, wz, vy), c1y = diff_of_products(wz, vx, wx, vz),
                    c1z = diff_of_products(wx, vy, wy, vx);
        const float c2x = diff_of_products(uy, wz, uz, wy), c2y = diff_of_products(uz, wx, ux, wz),
                    c2z = diff_of_products(ux, wy, uy, wx);
        const float a1 = __builtin_fmaf(c1x, nx, __builtin_fmaf(c1y, ny, c1z * nz));  // 2 area * |n| * b1
        const float a2 = __builtin_fmaf(c2x, nx, __builtin_fmaf(c2y, ny, c2z * nz));  // ... * b2
        const float a0 = l2 - a1 - a2;                                                // ... * b0
        const float ex1 = V[3 * i2] - V[3 * i1], ey1 = V[3 * i2 + 1] - V[3 * i1 + 1], ez1 = V[3 * i2 + 2] - V[3 * i1 + 2];
        const float e0 = sqrtf(__builtin_fmaf(ex1, ex1, __builtin_fmaf(ey1, ey1, ez1 * ez1)));  // edge opposite v0
        const float e1 = sqrtf(__builtin_fmaf(vx, vx, __builtin_fmaf(vy, vy, vz * vz)));        // opposite v1
        const float e2 = sqrtf(__builtin_fmaf(ux, ux, __builtin_fmaf(uy, uy, uz * uz)));        // opposite v2
        const float inv = on ? rsqrtf(l2) : 0.0f;
        // D = min over edges of b_i |n| / e_i = a_i / (|n| e_i)
        const float D = fminf(fminf(fmaxf(a0, 0.0f) / e0, fmaxf(a1, 0.0f) / e1), fmaxf(a2, 0.0f) / e2) * inv;
        on = on && D > 0.0f && isfinite(D);
        const float sc = on ? inv * D : 0.0f;
        nx *= sc; ny *= sc; nz *= sc;
    }
    const float r2 = rmax * rmax * 1.001f;
    cnt = 0;
#pragma unroll
    for (int j = 0; j < kBfCand; ++j) cand[j] = 0;
    uint64_t live = ballot(on);
    int stack = 0, sp = 0, node = 0;
    while (live != 0) {
        const BvhNode nd = load_node(nodes, node);
        const uint64_t h0 = ballot(box_dist2(px, py, pz, nd.lo0, nd.hi0) <= r2) & live;
        const uint64_t h1 = ballot(box_dist2(px, py, pz, nd.lo1, nd.hi1) <= r2) & live;
        int next = -1;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const uint64_t hm = c == 0 ? h0 : h1;
            if (hm == 0) continue;
            const int child = c == 0 ? nd.child0 : nd.child1;
            const int count = (c == 0 ? nd.count0 : nd.count1) & kCountMask;
            if (child < 0) {
                const bool in = __builtin_amdgcn_inverse_ballot_w64(hm);
                for (int k = 0; k < count; ++k) {
                    const int r = ~child + k;
                    const BvhTri tr = load_tri(tris, r);
                    if (in && tr.mesh == m && tr.id != t) {
                        const float lo[3] = {fminf(fminf(tr.v0[0], tr.v1[0]), tr.v2[0]),
                                             fminf(fminf(tr.v0[1], tr.v1[1]), tr.v2[1]),
                                             fminf(fminf(tr.v0[2], tr.v1[2]), tr.v2[2])};
                        const float hi[3] = {fmaxf(fmaxf(tr.v0[0], tr.v1[0]), tr.v2[0]),
                                             fmaxf(fmaxf(tr.v0[1], tr.v1[1]), tr.v2[1]),
                                             fmaxf(fmaxf(tr.v0[2], tr.v1[2]), tr.v2[2])};
                        if (box_dist2(px, py, pz, lo, hi) <= r2) {
#pragma unroll
                            for (int j = 0; j < kBfCand; ++j) cand[j] = j == cnt ? r : cand[j];
                            ++cnt;
                        }
                    }
                }
            } else if (next < 0) {
                next = child;
            } else {
                stack = lane == sp ? child : stack;
                ++sp;
            }
        }
        if (next < 0) {
            if (sp == 0) break;
            --sp;
            next = __builtin_amdgcn_readlane(stack, sp);
        }
        node = uniform(next);
    }
    if (!on || cnt > kBfCand) cnt = -1;
}

// 2^lg consecutive (sorted) points per wave, the other lanes idle.  A wave's radius queries
// walk the union of its points' neighbourhoods; when the points are few and sparse (a small
// session: a few thousand samples over a whole scene) that union spans most of the tree and
// a handful of such walks take the whole launch, so small launches spread their points over
// more waves.
constexpr int64_t kPrepWaves = 4096;  // 16 waves per CU

__host__ __device__ constexpr int prep_lanes_log2(int64_t n)
{
    int lg = 6;
    while (lg > 0 && (n >> lg) < kPrepWaves) --lg;
    return lg;
}

__global__ void __launch_bounds__(256) k_backface_prep(const float4* __restrict__ spos,
                                                       const int32_t* __restrict__ smesh, int64_t n,
                                                       const float* __restrict__ V, const int32_t* __restrict__ I,
                                                       const uint8_t* __restrict__ closed,
                                                       const BvhNode* __restrict__ nodes,
                                                       const BvhTri* __restrict__ tris, float rmax, int lg,
                                                       float4* __restrict__ bface, int32_t* __restrict__ bcand)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = (int)(g & 63);
    const int64_t i = lane < (1 << lg) ? ((g >> 6) << lg) + lane : n;  // n: an idle lane
    float4 p = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
    int m = -1;
    if (i < n) {
        p = spos[i];
        m = smesh[i];
    }
    float nx, ny, nz;
    int cnt, cand[kBfCand];
    backface_point(p.x, p.y, p.z, __float_as_int(p.w), m, i < n, V, I, closed, nodes, tris, rmax, nx, ny, nz, cnt,
                   cand);
    if (i < n) {
        bface[i] = make_float4(nx, ny, nz, __int_as_float(cnt));
#pragma unroll
        for (int j = 0; j < kBfCand; ++j)
            if (j < cnt) bcand[kBfCand * i + j] = cand[j];
    }
}

// May the stretch x + t (e - x), 0 <= t <= kEpsV, of a segment cross the triangle (v0,
// v1, v2) (x, y, z order)?  Watertight shear with x as origin, then "no" only when FP32
// rounding cannot explain the answer: some edge function clearly negative and another
// clearly positive (beyond 1e-4 of their magnitudes), or a parameter clearly outside
// [0, kEpsV] (beyond 1e-3 of kEpsV); a triangle nearly parallel to the segment may cross.
__device__ __forceinline__ bool stretch_may_cross(float xx, float xy, float xz, float ux, float uy, float uz,
                                                  const BvhTri& tr)
{
    const int kz = dominant_axis(ux, uy, uz);
    int kx, ky;
    cyclic_axes(kz, kx, ky);
    const float dkz = pick(kz, ux, uy, uz);
    const float sx = pick(kx, ux, uy, uz) / dkz, sy = pick(ky, ux, uy, uz) / dkz;
    const float o[3] = {xx, xy, xz};
    float X[3], Y[3], Z[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const float* q = v == 0 ? tr.v0 : (v == 1 ? tr.v1 : tr.v2);
        const float a = q[0] - o[0], b = q[1] - o[1], c = q[2] - o[2];
        const float ak = pick(kx, a, b, c), bk = pick(ky, a, b, c), ck = pick(kz, a, b, c);
        X[v] = __builtin_fmaf(-sx, ck, ak);
        Y[v] = __builtin_fmaf(-sy, ck, bk);
        Z[v] = ck;
    }
    const float U = X[2] * Y[1] - Y[2] * X[1];
    const float W1 = X[0] * Y[2] - Y[0] * X[2];
    const float W2 = X[1] * Y[0] - Y[1] * X[0];
    const float mag = fabsf(U) + fabsf(W1) + fabsf(W2);
    const float tol = 1e-4f * mag;
    const bool neg = fminf(fminf(U, W1), W2) < -tol, pos = fmaxf(fmaxf(U, W1), W2) > tol;
    if (neg && pos) return false;
    const float det = U + W1 + W2;
    if (!(fabsf(det) > 1e-5f * mag)) return true;
    const float T = __builtin_fmaf(W2, Z[2], __builtin_fmaf(W1, Z[1], U * Z[0]));
    const float tp = T / (det * dkz);
    return tp >= -1e-3f * kTlo && tp <= kTlo * 1.001f;
}

// The rule for the point x with back-face data (normal n scaled by the point's distance
// D to its triangle's edges, cnt neighbours cand[]) and eye e: true when the pair is
// occluded by the point's own closed mesh, whose bounding box is (lo, hi), without a
// traversal; segments longer than sqrt(l2max) are left to it.  The point is the FP32
// rounding of a point of its triangle and may lie off the plane by eta = 2^-24 (|x| + |y|
// + |z|); the segment then meets the plane within eta / c of x (c the cosine to the
// inward normal), inside the triangle while c D >= 4 eta, which the rule requires: so
// the segment does enter the solid through the triangle (or starts inside it).
template <class Cand>
__device__ __forceinline__ bool backface_rule(float nx, float ny, float nz, int cnt, const Cand& cand, float xx,
                                              float xy, float xz, float ex, float ey, float ez, float4 lo, float4 hi,
                                              float l2max, const BvhTri* __restrict__ tris)
{
    if (cnt < 0) return false;
    const float ux = ex - xx, uy = ey - xy, uz = ez - xz;
    const float l2 = __builtin_fmaf(ux, ux, __builtin_fmaf(uy, uy, uz * uz));
    const float dn = __builtin_fmaf(nx, ux, __builtin_fmaf(ny, uy, nz * uz));  // -c D |u|
    const float eta = 5.9604645e-8f * (fabsf(xx) + fabsf(xy) + fabsf(xz));
    if (!(dn < 0.0f && dn * dn >= 16.0f * eta * eta * l2 && l2 <= l2max)) return false;
    if (!(ex < lo.x || ex > hi.x || ey < lo.y || ey > hi.y || ez < lo.z || ez > hi.z)) return false;
    for (int j = 0; j < cnt; ++j)
        if (stretch_may_cross(xx, xy, xz, ux, uy, uz, load_tri_v(tris, cand(j)))) return false;
    return true;
}

// the rule for point i of a density launch (sorted order)
// The rule's buffers, copied to LDS once per work item and read back where the rule runs:
// the kernel arguments then need not stay in scalar registers across the whole kernel
// (which cost the posed-map kernel its register budget).
struct BfArgs {
    const float4* bface;
    const int32_t* bcand;
    const float4* mbox;
    const BvhTri* tris;
    float l2max;
};

template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T*)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ bool backface_occluded(const BfArgs& s_bf, const int32_t* smesh, int64_t i, float xx,
                                                  float xy, float xz, float ex, float ey, float ez)
{
    const float4* bface = uniform_ptr(s_bf.bface);
    const float4 bf = bface[i];
    const int c = __float_as_int(bf.w);
    if (c < 0) return false;
    const int m = smesh[i];
    const int32_t* cand = uniform_ptr(s_bf.bcand) + kBfCand * i;
    const float4* mbox = uniform_ptr(s_bf.mbox);
    return backface_rule(bf.x, bf.y, bf.z, c, [cand](int j) { return cand[j]; }, xx, xy, xz, ex, ey, ez,
                         mbox[2 * m], mbox[2 * m + 1],
                         __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(s_bf.l2max))),
                         uniform_ptr(s_bf.tris));
}

// Ray e + t d in the same sheared form as a segment with tmax = 1 (so s.tz = d[kz]).
__device__ __forceinline__ Seg make_ray(float ex, float ey, float ez, float dx, float dy, float dz, int kx, int ky,
                                        int kz)
{
    Seg s;
    s.ix = safe_inv(dx); s.iy = safe_inv(dy); s.iz = safe_inv(dz);
    s.qx = -ex * s.ix; s.qy = -ey * s.iy; s.qz = -ez * s.iz;
    s.kx = kx; s.ky = ky; s.kz = kz;
    const float dkz = pick(kz, dx, dy, dz);
    s.sx = pick(kx, dx, dy, dz) / dkz;
    s.sy = pick(ky, dx, dy, dz) / dkz;
    s.tz = dkz;
    return s;
}

// The watertight test of seg_tri returning the ray parameter of the hit,
// T' / (det d[kz]), or +inf when the ray misses the triangle's plane region (and for
// lanes with `active` false).  UNI as in seg_tri.
template <bool UNI>
__device__ __forceinline__ float ray_tri_t(const Seg& s, const TriEye& u, bool active)
{
    float akx, aky, akz, bkx, bky, bkz, ckx, cky, ckz;
    if (UNI) {
        akx = u.ax; aky = u.ay; akz = u.az;
        bkx = u.bx; bky = u.by; bkz = u.bz;
        ckx = u.cx; cky = u.cy; ckz = u.cz;
    } else {
        akx = pick(s.kx, u.ax, u.ay, u.az); aky = pick(s.ky, u.ax, u.ay, u.az); akz = pick(s.kz, u.ax, u.ay, u.az);
        bkx = pick(s.kx, u.bx, u.by, u.bz); bky = pick(s.ky, u.bx, u.by, u.bz); bkz = pick(s.kz, u.bx, u.by, u.bz);
        ckx = pick(s.kx, u.cx, u.cy, u.cz); cky = pick(s.ky, u.cx, u.cy, u.cz); ckz = pick(s.kz, u.cx, u.cy, u.cz);
    }
    const float Ax = __builtin_fmaf(-s.sx, akz, akx), Ay = __builtin_fmaf(-s.sy, akz, aky);
    const float Bx = __builtin_fmaf(-s.sx, bkz, bkx), By = __builtin_fmaf(-s.sy, bkz, bky);
    const float Cx = __builtin_fmaf(-s.sx, ckz, ckx), Cy = __builtin_fmaf(-s.sy, ckz, cky);
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    float lo = fminf(fminf(U, V), W), hi = fmaxf(fmaxf(U, V), W);
    const float amin = fminf(fminf(fabsf(U), fabsf(V)), fabsf(W));
    // the wave leaves when every active lane has edge functions of both signs, none zero
    if (ballot(active && !((lo * hi) * amin < 0.0f)) == 0) return INFINITY;
    if (active && amin == 0.0f) {
        asm volatile("" ::: "memory");
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
        lo = fminf(fminf(U, V), W);
        hi = fmaxf(fmaxf(U, V), W);
    }
    const bool mixed = (lo < 0.0f) && (hi > 0.0f);
    const float det = U + V + W;
    if (mixed || det == 0.0f) return INFINITY;
    const float Tp = __builtin_fmaf(W, ckz, __builtin_fmaf(V, bkz, U * akz));
    return Tp / (det * s.tz);
}

// Nearest surface along every lane's ray (lanes with `active`), tmin <= t < tbest on
// entry: the packet walk of occluded_packet, except that no lane stops early: each
// keeps its nearest hit and clips its box tests to it.  With UNI the rays share their
// axis order and direction signs: `nodes` is the node copy of octant `oct`, `tris` the
// record copy in the rays' axis order and (e0, e1, e2) the eye in that order;
// otherwise the plain node copy, the x, y, z record copy and the eye in x, y, z.
template <bool UNI>
__device__ void closest_packet(const BvhNode* __restrict__ nodes, const BvhTri* __restrict__ tris, float e0,
                               float e1, float e2, int oct, const Seg& sg, float tmin, bool active, float& tbest)
{
    const int lane = lane_id();
    const uint64_t live = ballot(active);
    if (live == 0) return;
    int stack = 0;
    int sp = 0;
    int node = 0;
    for (;;) {
        const BvhNode nd = load_node(nodes, node);
        const uint64_t h0 = ballot(UNI ? box_hit_signed(sg, nd.lo0, nd.hi0, tbest) : box_hit(sg, nd.lo0, nd.hi0, tbest)) & live;
        const uint64_t h1 = ballot(UNI ? box_hit_signed(sg, nd.lo1, nd.hi1, tbest) : box_hit(sg, nd.lo1, nd.hi1, tbest)) & live;
        const bool swap = (oct >> ((nd.count0 >> kSplitAxisShift) & 3)) & 1;
        int next = -1;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const bool first = (c == 0) != swap;
            const uint64_t m = first ? h0 : h1;
            if (m == 0) continue;
            const int child = first ? nd.child0 : nd.child1;
            const int count = (first ? nd.count0 : nd.count1) & kCountMask;
            if (child < 0) {
                const BvhTri* leaf = tris + (~child);
                BvhTri tr[kLeafMax];
#pragma unroll
                for (int k = 0; k < kLeafMax; ++k) tr[k] = load_tri(leaf, k);
                const bool in = __builtin_amdgcn_inverse_ballot_w64(m);
#pragma unroll
                for (int k = 0; k < kLeafMax; ++k) {
                    if (k >= count) break;
                    const float t = ray_tri_t<UNI>(sg, tri_eye(tr[k], e0, e1, e2), in);
                    if (in && t >= tmin && t < tbest) tbest = t;
                }
            } else if (next < 0) {
                next = child;
            } else {
                stack = lane == sp ? child : stack;
                ++sp;
            }
        }
        if (next < 0) {
            if (sp == 0) break;
            --sp;
            next = __builtin_amdgcn_readlane(stack, sp);
        }
        node = uniform(next);
    }
}

__device__ __forceinline__ unsigned long long to_fixed(float g, int shift)
{
    return (unsigned long long)ldexp((double)g, shift);
}

// ---------------------------------------------------------------------------
// a4: fixation records and the fixed-point scale
// ---------------------------------------------------------------------------
// a4: the record of fixation f; false (and a record that contributes nothing: zero
// gaze makes the gate s <= 0) for a non-finite eye or gaze, a zero gaze, or a
// duration that is negative, non-finite or above t_cap.
__device__ __forceinline__ bool fix_record_v(float ex, float ey, float ez, float rx, float ry, float rz, float t,
                                             double inv_norm, double kappa_scale, float t_cap, FixRec& r)
{
    // + 0: a -0 eye coordinate is stored as +0, so that e - x, whose sign the slab inverse
    // takes, is +0 whenever x equals the eye coordinate (the sign the packet's octant
    // classification gives a zero component)
    r.ex = ex + 0.0f; r.ey = ey + 0.0f; r.ez = ez + 0.0f;
    r.rx = rx; r.ry = ry; r.rz = rz;
    const double r2 = (double)r.rx * r.rx + (double)r.ry * r.ry + (double)r.rz * r.rz;
    const bool ok = isfinite(r.ex) && isfinite(r.ey) && isfinite(r.ez) && isfinite(r2) && r2 > 0.0 &&
                    isfinite(t) && t >= 0.0f && t <= t_cap;
    if (ok) {
        r.w = (float)((double)t * inv_norm);
        r.kappa = (float)(r2 * kappa_scale);
    } else {
        r.ex = r.ey = r.ez = 0.0f;
        r.rx = r.ry = r.rz = 0.0f;
        r.w = 0.0f;
        r.kappa = 1.0f;
    }
    return ok;
}

__device__ __forceinline__ bool fix_record(const float* __restrict__ eye, const float* __restrict__ gaze,
                                           const float* __restrict__ dur, int f, double inv_norm,
                                           double kappa_scale, float t_cap, FixRec& r)
{
    return fix_record_v(eye[3 * f], eye[3 * f + 1], eye[3 * f + 2], gaze[3 * f], gaze[3 * f + 1], gaze[3 * f + 2],
                        dur[f], inv_norm, kappa_scale, t_cap, r);
}

__global__ void k_fix_prep(const float* __restrict__ eye, const float* __restrict__ gaze,
                           const float* __restrict__ dur, int32_t F, double inv_norm, double kappa_scale,
                           FixRec* __restrict__ rec, unsigned int* __restrict__ wmax_bits)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    FixRec r;
    (void)fix_record(eye, gaze, dur, f, inv_norm, kappa_scale, INFINITY, r);
    rec[f] = r;
    atomicMax(wmax_bits, __float_as_uint(r.w));
}

// Records of one block of fixations added to an incremental map: the fixations whose
// start time lies in [t0, t1) (every fixation when `time` is NULL) are kept and
// written to rec[0 .. *kept) in no particular order (the map's sums are exact
// integers, so the order cannot change them).  A fixation is kept only if it is
// valid (a duration of at most 1e6 s) and its duration, rounded up to whole units of
// 2^-10 s, fits in what is left of the map's duration budget (budget[0] used,
// budget[1] total, in those units; a reservation that does not fit is returned, and
// 2^31 in-flight reservations of 2^30 units cannot wrap 64 bits); the others are counted
// in totals[1] (invalid) and totals[2] (over budget); totals[0] counts kept ones.
__global__ void k_fix_select(const float* __restrict__ eye, const float* __restrict__ gaze,
                             const float* __restrict__ dur, const double* __restrict__ time, int32_t F, double t0,
                             double t1, double inv_norm, double kappa_scale, FixRec* __restrict__ rec,
                             unsigned int* __restrict__ kept, unsigned long long* __restrict__ budget,
                             unsigned long long* __restrict__ totals)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    if (time) {
        const double t = time[f];
        if (!(t >= t0 && t < t1)) return;  // NaN times are outside every window
    }
    FixRec r;
    if (!fix_record(eye, gaze, dur, f, inv_norm, kappa_scale, 1.0e6f, r)) {
        atomicAdd(&totals[1], 1ull);
        return;
    }
    const unsigned long long units = (unsigned long long)ceil((double)dur[f] * 1024.0);
    const unsigned long long used = atomicAdd(&budget[0], units);
    if (used + units > budget[1]) {
        atomicAdd(&budget[0], 0ull - units);
        atomicAdd(&totals[2], 1ull);
        return;
    }
    rec[atomicAdd(kept, 1u)] = r;
    atomicAdd(&totals[0], 1ull);
}

__global__ void k_fix_shift(const unsigned int* __restrict__ wmax_bits, int32_t F, int32_t* __restrict__ shift)
{
    const float wmax = __uint_as_float(*wmax_bits);
    int e = 0;
    if (wmax > 0.0f) {
        (void)frexp((double)F * (double)wmax, &e);
        *shift = 62 - e;
    } else {
        *shift = 0;
    }
}

// Posed scenes.  pose [F][M][12]: row-major 3x4 (A | b) taking mesh m's own frame to
// the world at fixation f's time; A must be a similarity (rotation, optionally a
// reflection, times a uniform scale): s2 = trace(A^T A) / 3 and every entry of
// A^T A - s2 I within 1e-5 s2.  Seen from mesh m the fixation has eye
// A^-1 (e - b) and gaze A^-1 r (A^-1 = A^T / s2), each evaluated in FP64 in a fixed
// order and rounded to FP32: these are the inputs of the pair value in that frame,
// where angles, and so g, are those of the world.
__device__ __forceinline__ bool similarity(const float* __restrict__ P, double& s2)
{
    double G[3][3];
    bool ok = true;
    for (int k = 0; k < 12; ++k) ok = ok && isfinite(P[k]);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            G[i][j] = ((double)P[i] * (double)P[j] + (double)P[4 + i] * (double)P[4 + j]) +
                      (double)P[8 + i] * (double)P[8 + j];
    s2 = ((G[0][0] + G[1][1]) + G[2][2]) / 3.0;
    ok = ok && s2 > 0.0 && isfinite(s2);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) ok = ok && fabs(G[i][j] - (i == j ? s2 : 0.0)) <= 1e-5 * s2;
    return ok;
}

// (A^T v) / s2 with the columns of A taken in order
__device__ __forceinline__ void to_frame(const float* __restrict__ P, double s2, double v0, double v1, double v2,
                                         float& o0, float& o1, float& o2)
{
    o0 = (float)((((double)P[0] * v0 + (double)P[4] * v1) + (double)P[8] * v2) / s2);
    o1 = (float)((((double)P[1] * v0 + (double)P[5] * v1) + (double)P[9] * v2) / s2);
    o2 = (float)((((double)P[2] * v0 + (double)P[6] * v1) + (double)P[10] * v2) / s2);
}

// One thread per fixation: window, validity (the fixation's own and every mesh's
// pose), duration budget, then one record and one pose pair per mesh at the
// fixation's compacted index.
__global__ void k_fix_posed(const float* __restrict__ eye, const float* __restrict__ gaze,
                            const float* __restrict__ dur, const double* __restrict__ time,
                            const float* __restrict__ pose, int32_t F, int32_t M, int64_t stride, double t0,
                            double t1, double inv_norm, double kappa_scale, FixRec* __restrict__ rec,
                            float* __restrict__ xf, unsigned int* __restrict__ kept,
                            unsigned long long* __restrict__ budget, unsigned long long* __restrict__ totals)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    if (time) {
        const double t = time[f];
        if (!(t >= t0 && t < t1)) return;
    }
    FixRec r;
    bool ok = fix_record(eye, gaze, dur, f, inv_norm, kappa_scale, 1.0e6f, r);
    for (int m = 0; m < M && ok; ++m) {
        double s2;
        ok = similarity(pose + ((int64_t)f * M + m) * 12, s2);
    }
    if (!ok) {
        atomicAdd(&totals[1], 1ull);
        return;
    }
    const unsigned long long units = (unsigned long long)ceil((double)dur[f] * 1024.0);
    const unsigned long long used = atomicAdd(&budget[0], units);
    if (used + units > budget[1]) {
        atomicAdd(&budget[0], 0ull - units);
        atomicAdd(&totals[2], 1ull);
        return;
    }
    const unsigned idx = atomicAdd(kept, 1u);
    atomicAdd(&totals[0], 1ull);
    for (int m = 0; m < M; ++m) {
        const float* P = pose + ((int64_t)f * M + m) * 12;
        double s2;
        (void)similarity(P, s2);
        float ex, ey, ez, rx, ry, rz;
        to_frame(P, s2, (double)r.ex - (double)P[3], (double)r.ey - (double)P[7], (double)r.ez - (double)P[11], ex,
                 ey, ez);
        to_frame(P, s2, (double)r.rx, (double)r.ry, (double)r.rz, rx, ry, rz);
        FixRec rm;
        (void)fix_record_v(ex, ey, ez, rx, ry, rz, dur[f], inv_norm, kappa_scale, 1.0e6f, rm);
        rec[(int64_t)m * stride + idx] = rm;
        float* o = xf + ((int64_t)m * stride + idx) * 24;
        for (int k = 0; k < 12; ++k) o[k] = P[k];
        // inverse: A^T / s2 and -(A^T b) / s2
        for (int i = 0; i < 3; ++i) {
            o[12 + 4 * i + 0] = (float)((double)P[i] / s2);
            o[12 + 4 * i + 1] = (float)((double)P[4 + i] / s2);
            o[12 + 4 * i + 2] = (float)((double)P[8 + i] / s2);
        }
        float c0, c1, c2;
        to_frame(P, s2, (double)P[3], (double)P[7], (double)P[11], c0, c1, c2);
        o[15] = -c0; o[19] = -c1; o[23] = -c2;
    }
}

// ---------------------------------------------------------------------------
// The paper's visibility approximation (Sec. 3.2.2, Sec. 3.3.2, Appendix A)
// ---------------------------------------------------------------------------
// q v q^-1 for q = cos(a/2) + u sin(a/2), u a unit vector
__device__ __forceinline__ void quat_rotate(const double v[3], const double u[3], double a, double o[3])
{
    const double w = cos(0.5 * a), sn = sin(0.5 * a);
    const double q[3] = {sn * u[0], sn * u[1], sn * u[2]};
    const double t[3] = {2.0 * (q[1] * v[2] - q[2] * v[1]), 2.0 * (q[2] * v[0] - q[0] * v[2]),
                         2.0 * (q[0] * v[1] - q[1] * v[0])};
    o[0] = v[0] + w * t[0] + (q[1] * t[2] - q[2] * t[1]);
    o[1] = v[1] + w * t[1] + (q[2] * t[0] - q[0] * t[2]);
    o[2] = v[2] + w * t[2] + (q[0] * t[1] - q[1] * t[0]);
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// One thread per fixation, in FP64: the camera at the eye looking along the head
// direction (the gaze when no head direction is given) with the world's up (0, 1, 0)
// (or (0, 0, 1) for a vertical view); the crop of Appendix A on the near plane:
// the gaze turned by -+phi = -+atan(4 sigma) about u1 = r x i and u2 = r x u1 meets
// the plane at A0, A1, B0, B1, E is the gaze's own hit, a = |A1 - A0| / 2,
// b = |B1 - B0| / 2, alpha = angle of ME to the right vector, bounds E -+
// (sqrt(a^2 cos^2 + b^2 sin^2), sqrt(a^2 sin^2 + b^2 cos^2)).  The gate record keeps the
// eye, gaze and weight, with a cone (tan psi, psi the widest angle from the gaze to
// the crop's corners) that holds the whole cropped frustum.  A fixation whose crop
// is undefined (the cone reaches behind the camera) or whose corners lie 80 degrees
// or more off the gaze gets w = 0.
__global__ void k_zcam_prep(const float* __restrict__ eye, const float* __restrict__ gaze,
                            const float* __restrict__ dur, const float* __restrict__ head, int32_t F, double sigma,
                            double inv_norm, double widen, double near_, double far_, FixRec* __restrict__ rec,
                            ZCam* __restrict__ cam, unsigned int* __restrict__ wmax_bits)
{
    const int fi = blockIdx.x * blockDim.x + threadIdx.x;
    if (fi >= F) return;
    FixRec r;
    bool ok = fix_record(eye, gaze, dur, fi, inv_norm, 1.0, INFINITY, r);
    ZCam c;
    for (int k = 0; k < 3; ++k) c.x[k] = c.y[k] = c.f[k] = 0.0f;
    c.sx = c.sy = 1.0f; c.ox = c.oy = 0.0f; c.near_ = (float)near_; c.far_ = (float)far_; c.pad = 0.0f;
    double f[3] = {head ? head[3 * fi] : gaze[3 * fi], head ? head[3 * fi + 1] : gaze[3 * fi + 1],
                   head ? head[3 * fi + 2] : gaze[3 * fi + 2]};
    const double fn = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    ok = ok && isfinite(fn) && fn > 0.0;
    double tanpsi = 0.0;
    if (ok) {
        for (int k = 0; k < 3; ++k) f[k] /= fn;
        const double up0[3] = {0.0, 1.0, 0.0}, up1[3] = {0.0, 0.0, 1.0};
        const double* up = fabs(f[1]) < 1.0 - 1e-6 ? up0 : up1;
        double x[3], y[3];
        cross3(f, up, x);
        const double xn = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        for (int k = 0; k < 3; ++k) x[k] /= xn;
        cross3(x, f, y);
        const double g[3] = {r.rx, r.ry, r.rz};
        double rc[3] = {g[0] * x[0] + g[1] * x[1] + g[2] * x[2], g[0] * y[0] + g[1] * y[1] + g[2] * y[2],
                        -(g[0] * f[0] + g[1] * f[1] + g[2] * f[2])};
        const double rn = sqrt(rc[0] * rc[0] + rc[1] * rc[1] + rc[2] * rc[2]);
        for (int k = 0; k < 3; ++k) rc[k] /= rn;
        const double phi = atan(4.0 * sigma);
        const double ifw[3] = {0.0, 0.0, -1.0}, jr[3] = {1.0, 0.0, 0.0};
        double u1[3], u2[3];
        cross3(rc, ifw, u1);
        double n1 = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
        if (n1 < 1e-12) {
            cross3(rc, jr, u1);
            n1 = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
        }
        for (int k = 0; k < 3; ++k) u1[k] /= n1;
        cross3(rc, u1, u2);
        const double n2 = sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
        for (int k = 0; k < 3; ++k) u2[k] /= n2;
        double a0[3], a1[3], b0[3], b1[3];
        quat_rotate(rc, u1, -phi, a0); quat_rotate(rc, u1, phi, a1);
        quat_rotate(rc, u2, -phi, b0); quat_rotate(rc, u2, phi, b1);
        ok = rc[2] < 0.0 && a0[2] < 0.0 && a1[2] < 0.0 && b0[2] < 0.0 && b1[2] < 0.0;
        if (ok) {
            const double A0x = -near_ / a0[2] * a0[0], A0y = -near_ / a0[2] * a0[1];
            const double A1x = -near_ / a1[2] * a1[0], A1y = -near_ / a1[2] * a1[1];
            const double B0x = -near_ / b0[2] * b0[0], B0y = -near_ / b0[2] * b0[1];
            const double B1x = -near_ / b1[2] * b1[0], B1y = -near_ / b1[2] * b1[1];
            const double Ex = -near_ / rc[2] * rc[0], Ey = -near_ / rc[2] * rc[1];
            const double a = sqrt((A1x - A0x) * (A1x - A0x) + (A1y - A0y) * (A1y - A0y)) / 2.0;
            const double b = sqrt((B1x - B0x) * (B1x - B0x) + (B1y - B0y) * (B1y - B0y)) / 2.0;
            const double me = sqrt(Ex * Ex + Ey * Ey);
            const double al = me > 0.0 ? acos(fmax(-1.0, fmin(1.0, Ex / me))) : 0.0;
            const double ca = cos(al), sa = sin(al);
            const double hx = sqrt(a * a * ca * ca + b * b * sa * sa), hy = sqrt(a * a * sa * sa + b * b * ca * ca);
            const double l = Ex - hx, rr = Ex + hx, bt = Ey - hy, tp = Ey + hy;
            // the widest angle from the gaze to a corner of the crop
            double cmin = 1.0;
            for (int k = 0; k < 4; ++k) {
                const double cx = (k & 1) ? rr : l, cy = (k & 2) ? tp : bt;
                const double cl = sqrt(cx * cx + cy * cy + near_ * near_);
                cmin = fmin(cmin, (cx * rc[0] + cy * rc[1] - near_ * rc[2]) / cl);
            }
            ok = cmin > 0.17364817766693033;  // cos 80 degrees
            tanpsi = ok ? sqrt(1.0 - cmin * cmin) / cmin : 0.0;
            for (int k = 0; k < 3; ++k) {
                c.x[k] = (float)x[k]; c.y[k] = (float)y[k]; c.f[k] = (float)f[k];
            }
            c.sx = (float)(2.0 * near_ / (rr - l));
            c.ox = (float)((rr + l) / (rr - l));
            c.sy = (float)(2.0 * near_ / (tp - bt));
            c.oy = (float)((tp + bt) / (tp - bt));
        }
    }
    if (ok) {
        const double r2 = (double)r.rx * r.rx + (double)r.ry * r.ry + (double)r.rz * r.rz;
        r.kappa = (float)(r2 * (1.0 - widen) / (1.0 + tanpsi * tanpsi));
    } else {
        r.ex = r.ey = r.ez = 0.0f;
        r.rx = r.ry = r.rz = 0.0f;
        r.w = 0.0f;
        r.kappa = 1.0f;
    }
    rec[fi] = r;
    cam[fi] = c;
    atomicMax(wmax_bits, __float_as_uint(r.w));
}

// One wave per 8 x 8 block of pixels of one fixation's z-buffer: the ray through
// each pixel centre, direction x' right + y' up + forward (so the ray parameter is
// the depth), x' = (x_ndc + ox) / sx; the buffer keeps the nearest hit with depth in
// [near, far], +inf where there is none.  Fixations with w = 0 get +inf everywhere.
__global__ void __launch_bounds__(256, 8) k_zbuffer(const BvhNode* __restrict__ nodes, int64_t node_stride,
                                                 const BvhTri* __restrict__ tris, int64_t tri_stride,
                                                 const FixRec* __restrict__ rec, const ZCam* __restrict__ cams,
                                                 int32_t F, int32_t R, float* __restrict__ zbuf)
{
    const int lane = lane_id();
    const int64_t blocks_per_fix = (int64_t)(R / 8) * (R / 8);
    const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= blocks_per_fix * F) return;
    const int f = (int)(item / blocks_per_fix);
    const int blk = (int)(item % blocks_per_fix);
    const int i = (blk % (R / 8)) * 8 + (lane & 7);
    const int j = (blk / (R / 8)) * 8 + (lane >> 3);
    const FixRec fr = load_fix(rec, f);
    const ZCam c = cams[f];
    float tbest = c.far_;
    const bool active = fr.w > 0.0f;
    if (uniform(active ? 1 : 0)) {
        const float nx = -1.0f + (2.0f * i + 1.0f) / (float)R, ny = -1.0f + (2.0f * j + 1.0f) / (float)R;
        const float xc = (nx + c.ox) / c.sx, yc = (ny + c.oy) / c.sy;
        const float dx = __builtin_fmaf(xc, c.x[0], __builtin_fmaf(yc, c.y[0], c.f[0]));
        const float dy = __builtin_fmaf(xc, c.x[1], __builtin_fmaf(yc, c.y[1], c.f[1]));
        const float dz = __builtin_fmaf(xc, c.x[2], __builtin_fmaf(yc, c.y[2], c.f[2]));
        tbest = nextafterf(c.far_, INFINITY);
        // the 64 rays of a block share the forward axis' dominant axis as their shear axis
        // and their direction signs when each keeps 0.4 of its length along it (as the
        // segments of packet_visibility); then they read the octant node copy and the
        // record copy in that axis order
        const float afx = fabsf(c.f[0]), afy = fabsf(c.f[1]), afz = fabsf(c.f[2]);
        const int kz = uniform(afx > afy ? (afx > afz ? 0 : 2) : (afy > afz ? 1 : 2));
        const int kx = kz == 2 ? 0 : kz + 1;
        const int ky = kx == 2 ? 0 : kx + 1;
        const float dk = pick(kz, dx, dy, dz);
        const uint64_t neg_x = ballot(signbit(dx)), neg_y = ballot(signbit(dy)), neg_z = ballot(signbit(dz));
        const bool shared = ballot(!(dk * dk >= 0.16f * (dx * dx + dy * dy + dz * dz))) == 0 &&
                            (neg_x == 0 || ~neg_x == 0) && (neg_y == 0 || ~neg_y == 0) && (neg_z == 0 || ~neg_z == 0);
        if (shared) {
            const int oct = (neg_x != 0 ? 1 : 0) | (neg_y != 0 ? 2 : 0) | (neg_z != 0 ? 4 : 0);
            const Seg sg = make_ray(fr.ex, fr.ey, fr.ez, dx, dy, dz, kx, ky, kz);
            closest_packet<true>(nodes + oct * node_stride, tris + kz * tri_stride, pick(kx, fr.ex, fr.ey, fr.ez),
                                 pick(ky, fr.ex, fr.ey, fr.ez), pick(kz, fr.ex, fr.ey, fr.ez), oct, sg, c.near_,
                                 true, tbest);
        } else {
            int lx, ly, lz;
            axis_order(dx, dy, dz, lx, ly, lz);
            const Seg sg = make_ray(fr.ex, fr.ey, fr.ez, dx, dy, dz, lx, ly, lz);
            const int lead = 0;
            const int oct = (int)(__shfl(dx, lead) < 0.0f) | ((int)(__shfl(dy, lead) < 0.0f) << 1) |
                            ((int)(__shfl(dz, lead) < 0.0f) << 2);
            closest_packet<false>(nodes, tris + 2 * tri_stride, fr.ex, fr.ey, fr.ez, uniform(oct), sg, c.near_, true,
                                  tbest);
        }
        if (!(tbest <= c.far_)) tbest = INFINITY;
    } else {
        tbest = INFINITY;
    }
    zbuf[((int64_t)f * R + j) * R + i] = tbest;
}

// ---------------------------------------------------------------------------
// spatial order: 7-bit-per-axis Morton buckets, counting sort
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t spread3(uint32_t v)
{
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void k_morton(const float* __restrict__ pos, int64_t n, float lox, float loy, float loz, float inv_cell,
                         int cells, uint32_t* __restrict__ key, uint32_t* __restrict__ hist)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float fx = (pos[3 * i] - lox) * inv_cell, fy = (pos[3 * i + 1] - loy) * inv_cell,
                fz = (pos[3 * i + 2] - loz) * inv_cell;
    const uint32_t cx = (uint32_t)min(max((int)fx, 0), cells - 1);
    const uint32_t cy = (uint32_t)min(max((int)fy, 0), cells - 1);
    const uint32_t cz = (uint32_t)min(max((int)fz, 0), cells - 1);
    const uint32_t k = spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2);
    key[i] = k;
    atomicAdd(&hist[k], 1u);
}

__global__ void k_scatter(const float* __restrict__ pos, const int32_t* __restrict__ tri,
                          const int32_t* __restrict__ mesh, const int32_t* __restrict__ tri_mesh, int64_t T, int64_t n,
                          const uint32_t* __restrict__ key, uint32_t* __restrict__ cursor, float4* __restrict__ spos,
                          int32_t* __restrict__ smesh, int32_t* __restrict__ inv, int32_t base)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t dst = atomicAdd(&cursor[key[i]], 1u);
    int32_t t = tri ? tri[i] : -1;
    if (t < 0 || t >= T) t = -1;  // unknown triangle: no own-triangle exclusion
    const int32_t m = mesh ? mesh[i] : (t >= 0 ? tri_mesh[t] : -1);
    spos[dst] = make_float4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], __int_as_float(t));
    smesh[dst] = m;
    inv[i] = base + (int32_t)dst;  // where input point i sits in sorted order (written in input order)
}

// ---------------------------------------------------------------------------
// a5 + a6: gate, exact value, visibility, fixed-point accumulation
// ---------------------------------------------------------------------------
// Visibility of the wave's slots that need it, for one fixation, in one frame: the
// segments run between the points p[k] and the eye (ex, ey, ez), both in the frame of
// the BVH whose octant node copies start at `nodes` (node_stride nodes apart) and
// whose axis-permuted record copies start at `tris` (tri_stride records apart).
template <int SPL>
__device__ __forceinline__ void packet_visibility(const BvhNode* __restrict__ nodes, int64_t node_stride,
                                                  const BvhTri* __restrict__ tris, int64_t tri_stride, float ex,
                                                  float ey, float ez, float rx, float ry, float rz,
                                                  const float4 (&p)[SPL], const int (&otri)[SPL],
                                                  const int (&omesh)[SPL], int mode, const bool (&need)[SPL],
                                                  bool (&occl)[SPL], TravCount& n_visits)
{
    // Every lane shears along segment_axis: the gaze's dominant axis for every in-cone
    // segment at the cone angles in use.  When all of the packet's segments take it and
    // share their direction signs, the packet reads the record copy permuted into that
    // order and the node copy of its octant (no per-lane permutation or min/max).
    const int gz = uniform(dominant_axis(rx, ry, rz));
    int gx, gy;
    cyclic_axes(gz, gx, gy);
    bool shared = true;
    // per axis: lanes with a segment (any slot) running from the eye towards -axis / +axis.
    // An exactly zero component counts as -axis here: the segment then runs towards +axis
    // for the node copy, as its slab inverse (+1e30 for the +0 of e - x) does; counted by its
    // sign bit, a +0 would pick the copy stored for the other direction, whose boxes that
    // lane could miss.
    uint64_t nx_m = 0, ny_m = 0, nz_m = 0, px_m = 0, py_m = 0, pz_m = 0;
    int kz[SPL];
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
        const float dx = p[k].x - ex, dy = p[k].y - ey, dz = p[k].z - ez;
        kz[k] = segment_axis(gz, dx, dy, dz);
        shared = shared && (!need[k] || kz[k] == gz);
        nx_m |= ballot(need[k] && dx <= 0.0f);
        ny_m |= ballot(need[k] && dy <= 0.0f);
        nz_m |= ballot(need[k] && dz <= 0.0f);
        px_m |= ballot(need[k] && dx > 0.0f);
        py_m |= ballot(need[k] && dy > 0.0f);
        pz_m |= ballot(need[k] && dz > 0.0f);
    }
    // ... and every segment of every slot has the same direction signs
    shared = ballot(!shared) == 0 && (nx_m == 0 || px_m == 0) && (ny_m == 0 || py_m == 0) &&
             (nz_m == 0 || pz_m == 0);
    Seg sg[SPL];
    float org[SPL][3];
    if (shared) {
#pragma unroll
        for (int k = 0; k < SPL; ++k) {
            sg[k] = make_seg(p[k].x, p[k].y, p[k].z, ex, ey, ez, gx, gy, gz);
            org[k][0] = pick(gx, p[k].x, p[k].y, p[k].z);
            org[k][1] = pick(gy, p[k].x, p[k].y, p[k].z);
            org[k][2] = pick(gz, p[k].x, p[k].y, p[k].z);
        }
        // eye-to-point octant (child order); the segments run the other way (node copy)
        const int oct = (nx_m != 0 ? 1 : 0) | (ny_m != 0 ? 2 : 0) | (nz_m != 0 ? 4 : 0);
        occluded_packet<SPL, true>(nodes + (oct ^ 7) * node_stride, tris + gz * tri_stride, org, oct, sg, otri,
                                   omesh, mode, need, occl, n_visits);
    } else {
#pragma unroll
        for (int k = 0; k < SPL; ++k) {
            int lx, ly;
            cyclic_axes(kz[k], lx, ly);
            sg[k] = make_seg(p[k].x, p[k].y, p[k].z, ex, ey, ez, lx, ly, kz[k]);
            org[k][0] = p[k].x; org[k][1] = p[k].y; org[k][2] = p[k].z;
        }
        // child order from one lane's octant (the order affects speed, not results)
        const int lead = __builtin_ctzll(nx_m | px_m);
        const int oct = (int)((nx_m >> lead) & 1) | (int)(((ny_m >> lead) & 1) << 1) | (int)(((nz_m >> lead) & 1) << 2);
        occluded_packet<SPL, false>(nodes, tris + 2 * tri_stride, org, oct, sg, otri, omesh, mode, need, occl,
                                    n_visits);
    }
}

// The pair under the paper's approximation: inside the fixation's cropped frustum
// (n <= D <= f, |x_ndc| <= 1, |y_ndc| <= 1, D the depth along the camera's forward
// axis) and passing the depth test D - zbuf(pixel) <= eps D, the angular Gaussian
// of Sec. 3.2.1 (not cut at 4 sigma: the frustum does the cutting); else 0.
// `in` reports whether the point lies in the frustum.
__device__ __forceinline__ float zb_value(float x, float y, float z, const FixRec& fr, const ZCam& c,
                                          const float* __restrict__ zb, int R, float eps, float kexp, bool& in)
{
    float phx, plx, phy, ply, phz, plz;
    two_sum(x, -fr.ex, phx, plx);
    two_sum(y, -fr.ey, phy, ply);
    two_sum(z, -fr.ez, phz, plz);
    const float xc = __builtin_fmaf(phx, c.x[0], __builtin_fmaf(phy, c.x[1], __builtin_fmaf(phz, c.x[2],
                     __builtin_fmaf(plx, c.x[0], __builtin_fmaf(ply, c.x[1], plz * c.x[2])))));
    const float yc = __builtin_fmaf(phx, c.y[0], __builtin_fmaf(phy, c.y[1], __builtin_fmaf(phz, c.y[2],
                     __builtin_fmaf(plx, c.y[0], __builtin_fmaf(ply, c.y[1], plz * c.y[2])))));
    const float D = __builtin_fmaf(phx, c.f[0], __builtin_fmaf(phy, c.f[1], __builtin_fmaf(phz, c.f[2],
                    __builtin_fmaf(plx, c.f[0], __builtin_fmaf(ply, c.f[1], plz * c.f[2])))));
    in = false;
    if (!(D >= c.near_ && D <= c.far_)) return 0.0f;
    const float nx = c.sx * xc / D - c.ox, ny = c.sy * yc / D - c.oy;
    if (!(fabsf(nx) <= 1.0f && fabsf(ny) <= 1.0f)) return 0.0f;
    in = true;
    const int i = min(R - 1, max(0, (int)floorf((nx + 1.0f) * 0.5f * (float)R)));
    const int j = min(R - 1, max(0, (int)floorf((ny + 1.0f) * 0.5f * (float)R)));
    const float depth = zb[(int64_t)j * R + i];
    if (D - depth > eps * D) return 0.0f;
    const float cx = diff_of_products(phy, fr.rz, phz, fr.ry) + (ply * fr.rz - plz * fr.ry);
    const float cy = diff_of_products(phz, fr.rx, phx, fr.rz) + (plz * fr.rx - plx * fr.rz);
    const float cz = diff_of_products(phx, fr.ry, phy, fr.rx) + (plx * fr.ry - ply * fr.rx);
    const float q = __builtin_fmaf(cx, cx, __builtin_fmaf(cy, cy, cz * cz));
    const float lo = __builtin_fmaf(plx, fr.rx, __builtin_fmaf(ply, fr.ry, plz * fr.rz));
    const float d1 = __builtin_fmaf(phx, fr.rx, __builtin_fmaf(phy, fr.ry, __builtin_fmaf(phz, fr.rz, lo)));
    if (!(d1 > 0.0f)) return 0.0f;
    return fr.w * exp2f(-(q / (d1 * d1)) * kexp);
}

// One work item of the density map: the samples of one tile (256 * SPL consecutive
// sorted samples) against one chunk of the fixations, by the whole workgroup.
// OCC = 0: no occlusion (no traversal code); OCC = 1: visibility by the BVH when
// a.occ_mode != 0.  FB: fixations staged in LDS per round.
template <int SPL, int OCC, int FB, bool INST = false, bool ZB = false>
__device__ __forceinline__ void density_item(const DensityLaunch& a, int64_t tile, int chunk, int F)
{
    // per fixation of the block, 48 bytes: (rx, ry, rz, c0), (ax, ay, az, cc), (-kappa, -, -, -);
    // one base address reaches all three with immediate offsets.  kGateGroup - 1 entries past
    // the block's last fixation never pass the gate, so the gate takes fixations in groups.
    constexpr int kGateGroup = OCC != 0 ? 1 : 4;  // fixations per gate test (one where registers are tight)
    __shared__ float4 s_co[3 * (FB + kGateGroup - 1)];
    __shared__ unsigned long long s_acc[kThreads * SPL];  // one entry per sample, owned by one lane
    __shared__ float s_rad;
    __shared__ uint32_t s_stats[kDensityStats];
    __shared__ uint32_t s_keep[kThreads / 64];  // fixations of the block kept by each staging wave
    __shared__ BfArgs s_bf;                      // the back-face rule's buffers

    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int64_t tile_base = tile * (int64_t)(kThreads * SPL);
    const int64_t wave_base = tile_base + wave * (64 * SPL);
    const int64_t n = a.n;

    // tile origin: its first sample; radius: largest distance of a tile sample to it
    const float4 o4 = a.spos[tile_base];
    if (threadIdx.x == 0) s_rad = 0.0f;
    if (threadIdx.x < kDensityStats) s_stats[threadIdx.x] = 0u;
    if (OCC != 0 && !ZB && threadIdx.x == 0) s_bf = BfArgs{a.bface, a.bcand, a.mbox, a.bf_tris, a.bf_L2max};
    __syncthreads();
    uint32_t n_in = 0, n_vis = 0, n_trav = 0, n_bf = 0;  // wave-uniform counters
    TravCount n_visits;

    float px[SPL], py[SPL], pz[SPL], pq[SPL];
    float rad = 0.0f;
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
        const int64_t i = wave_base + k * 64 + lane;
        const float4 p = i < n ? a.spos[i] : o4;
        px[k] = p.x - o4.x; py[k] = p.y - o4.y; pz[k] = p.z - o4.z;
        pq[k] = __builtin_fmaf(px[k], px[k], __builtin_fmaf(py[k], py[k], pz[k] * pz[k]));
        rad = fmaxf(rad, pq[k]);
        s_acc[wave * (64 * SPL) + k * 64 + lane] = 0ull;
    }
    atomicMax((unsigned int*)&s_rad, __float_as_uint(rad));
    __syncthreads();
    // eyes within 2 tile radii of the origin take the exact path for every pair
    const float near2 = 4.0f * s_rad + 1e-12f;

    const int shift = *a.fx_shift;
    const int f_begin = chunk * a.fix_per_chunk;
    // wave-uniform bounds in scalar registers (F may come from a vector load of the live
    // count): the fixation loop then counts in scalar instructions
    const int f_end = uniform(min(F, f_begin + a.fix_per_chunk));

    for (int fb = f_begin; fb < f_end; fb += FB) {
        const int nbf = uniform(min(FB, f_end - fb));
        __syncthreads();
        // Staging, one thread per fixation of the block.  Only fixations whose gate cone
        // can reach the tile are kept (listed in order, with their index): a sample x
        // passes the gate iff the angle between r and x - e is below psi_g, cos^2 psi_g =
        // kappa / |r|^2, and every sample lies within rad_t of the origin o, so the tile
        // can hold a passing sample only if angle(r, o - e) < psi_g + delta, sin delta =
        // rad_t / |o - e|.  The test adds 1e-4 rad to that angle, far above the FP32
        // error of the gate itself, so every fixation that the per-sample gate would pass
        // for some sample of the tile is kept; the others could only be skipped there.
        bool keep = false;
        if (threadIdx.x < nbf) {
            const FixRec fr = a.fix[fb + threadIdx.x];
            const float ex = fr.ex - o4.x, ey = fr.ey - o4.y, ez = fr.ez - o4.z;
            const float e2 = __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez));
            const float c0 = -__builtin_fmaf(fr.rx, ex, __builtin_fmaf(fr.ry, ey, fr.rz * ez));
            if (fr.w > 0.0f) {  // zero weight: contributes nothing anywhere
                // the tile's bounding radius about its origin, rounded up
                const float rad_t = __builtin_fmaf(sqrtf(s_rad), 1.001f, 1e-6f);
                const float rr = __builtin_fmaf(fr.rx, fr.rx, __builtin_fmaf(fr.ry, fr.ry, fr.rz * fr.rz));
                const float cg2 = fminf(fr.kappa / rr, 1.0f);
                const float cg = sqrtf(cg2), sg = sqrtf(1.0f - cg2);
                const float sd = fminf(rad_t * __frsqrt_rn(e2), 1.0f);
                const float cd = sqrtf(fmaxf(1.0f - sd * sd, 0.0f));
                const float cA = cg * cd - sg * sd, sA = sg * cd + cg * sd;  // cos, sin (psi_g + delta)
                const float cT = __builtin_fmaf(-1e-4f, sA, cA);            // cos (psi_g + delta + 1e-4)
                keep = e2 <= near2 || !(cT > 0.0f) || (c0 > 0.0f && c0 * c0 > cT * cT * rr * e2);
            }
        }
        // the kept fixations in block order: a wave-level prefix, then the waves in order
        const uint64_t kb = ballot(keep);
        if (lane == 0) s_keep[wave] = (uint32_t)__popcll(kb);
        __syncthreads();
        uint32_t pos = (uint32_t)__popcll(kb & ((1ull << lane) - 1ull)), nb_all = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            const uint32_t c = s_keep[w];
            pos += w < wave ? c : 0u;
            nb_all += c;
        }
        const int nb = uniform((int)nb_all);
        if (keep) {
            // the record again (a cached reload: fewer registers held across the barrier)
            const int fidx = fb + threadIdx.x;
            const FixRec fr = a.fix[fidx];
            const float ex = fr.ex - o4.x, ey = fr.ey - o4.y, ez = fr.ez - o4.z;
            const float e2 = __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez));
            const float k = fr.kappa;
            const float c0 = -__builtin_fmaf(fr.rx, ex, __builtin_fmaf(fr.ry, ey, fr.rz * ez));
            // an eye within 2 tile radii: s > 0 for every sample of the tile
            const float cc = e2 <= near2 ? 3.0e38f : -k * e2;
            s_co[3 * pos] = make_float4(fr.rx, fr.ry, fr.rz, c0);
            s_co[3 * pos + 1] = make_float4(2.0f * k * ex, 2.0f * k * ey, 2.0f * k * ez, cc);
            s_co[3 * pos + 2] = make_float4(-k, __int_as_float(fidx), 0.0f, 0.0f);
        }
        if (threadIdx.x < kGateGroup - 1) {
            // s = 0 * |0| + (-3e38) < 0 at every point: never a candidate
            s_co[3 * (nb + threadIdx.x)] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            s_co[3 * (nb + threadIdx.x) + 1] = make_float4(0.0f, 0.0f, 0.0f, -3.0e38f);
            s_co[3 * (nb + threadIdx.x) + 2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        if (threadIdx.x == 0) s_stats[6] += (uint32_t)nb;  // only thread 0 writes it until the end
        __syncthreads();
        for (int jg = 0; jg < nb; jg += kGateGroup) {
            // the gate of kGateGroup fixations, one wave mask per fixation and slot; a group
            // with no candidate costs one scalar test
            uint64_t gm[kGateGroup][SPL];
            uint64_t gany = 0;
#pragma unroll
            for (int h = 0; h < kGateGroup; ++h) {
                const float4 ra = s_co[3 * (jg + h)];
                const float4 rb = s_co[3 * (jg + h) + 1];
                const float nk = s_co[3 * (jg + h) + 2].x;
#pragma unroll
                for (int k = 0; k < SPL; ++k) {
                    float d = __builtin_fmaf(ra.x, px[k], ra.w);
                    d = __builtin_fmaf(ra.y, py[k], d);
                    d = __builtin_fmaf(ra.z, pz[k], d);
                    float m = __builtin_fmaf(rb.x, px[k], rb.w);
                    m = __builtin_fmaf(rb.y, py[k], m);
                    m = __builtin_fmaf(rb.z, pz[k], m);
                    m = __builtin_fmaf(nk, pq[k], m);
                    const float sv = __builtin_fmaf(d, fabsf(d), m);
                    gm[h][k] = ballot(sv > 0.0f);
                    gany |= gm[h][k];
                }
            }
            if (gany == 0) continue;
#pragma unroll 1
            for (int h = 0; h < kGateGroup; ++h) {
                uint64_t cm[SPL];
                uint64_t cany = 0;
#pragma unroll
                for (int k = 0; k < SPL; ++k) {
                    // a uniform select, not an index into gm (which would put it in memory)
                    cm[k] = gm[0][k];
#pragma unroll
                    for (int hh = 1; hh < kGateGroup; ++hh) cm[k] = h == hh ? gm[hh][k] : cm[k];
                    cany |= cm[k];
                }
                if (cany == 0) continue;

                // exact path for this fixation: values of the passing slots, then one packet
                // traversal for every slot that needs a visibility answer
                const int f = uniform(__float_as_int(s_co[3 * (jg + h) + 2].y));
                const FixRec fr = load_fix(a.fix, f);
                float g[SPL];
                float4 p[SPL];
                bool need[SPL];
                bool any_need = false;
                ZCam zc;
                if (ZB) zc = reinterpret_cast<const ZCam*>(a.zcam)[f];
#pragma unroll
                for (int k = 0; k < SPL; ++k) {
                    const int64_t i = wave_base + k * 64 + lane;
                    const bool c = __builtin_amdgcn_inverse_ballot_w64(cm[k]) && i < n;
                    g[k] = 0.0f;
                    p[k] = make_float4(fr.ex, fr.ey, fr.ez, __int_as_float(-1));
                    bool in = false;
                    if (ballot(c) != 0 && c) {
                        p[k] = a.spos[i];
                        if (ZB)
                            g[k] = zb_value(p[k].x, p[k].y, p[k].z, fr, zc, a.zbuf + (int64_t)f * a.zres * a.zres, a.zres,
                                            a.zeps, a.kexp, in);
                        else
                            g[k] = pair_value(p[k].x, p[k].y, p[k].z, fr.ex, fr.ey, fr.ez, fr.rx, fr.ry, fr.rz, fr.w,
                                              a.cone2, a.kexp);
                    }
                    need[k] = OCC != 0 && a.occ_mode != 0 && g[k] > 0.0f;
                    any_need = any_need || need[k];
                    n_in += (uint32_t)__popcll(ballot(ZB ? in : g[k] > 0.0f));
                }
                bool occl[SPL];
#pragma unroll
                for (int k = 0; k < SPL; ++k) occl[k] = false;
                if (OCC != 0 && !ZB && a.bface && ballot(any_need) != 0) {
                    // the back-face rule first: pairs it settles leave the packet (posed
                    // launches: sample and eye in the sample's own mesh frame)
                    any_need = false;
#pragma unroll
                    for (int k = 0; k < SPL; ++k) {
                        const int64_t i = wave_base + k * 64 + lane;
                        if (need[k] &&
                            backface_occluded(s_bf, a.smesh, i, p[k].x, p[k].y, p[k].z, fr.ex, fr.ey, fr.ez)) {
                            need[k] = false;
                            occl[k] = true;
                        }
                        n_bf += (uint32_t)__popcll(ballot(occl[k]));
                        any_need = any_need || need[k];
                    }
                }
                if (OCC != 0 && ballot(any_need) != 0) {
                    int otri[SPL], omesh[SPL];
#pragma unroll
                    for (int k = 0; k < SPL; ++k) {
                        const int64_t i = wave_base + k * 64 + lane;
                        otri[k] = need[k] ? __float_as_int(p[k].w) : -1;
                        omesh[k] = need[k] ? a.smesh[i] : -1;
                    }
                    if (!INST) {
                        // the walk answers the lanes it tests; lanes the back-face rule settled keep it
                        bool o1[SPL];
                        packet_visibility<SPL>(a.nodes, a.node_stride, a.tris, a.tri_stride, fr.ex, fr.ey, fr.ez, fr.rx,
                                               fr.ry, fr.rz, p, otri, omesh, a.occ_mode, need, o1, n_visits);
#pragma unroll
                        for (int k = 0; k < SPL; ++k) occl[k] = occl[k] || o1[k];
                        ++n_trav;
                    } else {
                        // One BVH per mesh.  Static scenes (xf NULL): every mesh in the world
                        // frame, the segments as they are.  Posed launches: every mesh in its
                        // own frame at this fixation's time; the points move with their mesh
                        // (forward pose of this launch's mesh), then into the occluding mesh's
                        // frame (its inverse pose), whose eye and gaze are that mesh's fixation
                        // record; tau is unchanged by the (affine) change of frame.  With
                        // GM_OCC_SELF a lane takes part only in its own mesh.
                        const bool moving = a.xf != nullptr;
                        const float* fw = moving ? a.xf + ((int64_t)a.self_mesh * a.fix_stride + f) * 24 : nullptr;
                        for (int mi = 0; mi < a.n_inst; ++mi) {
                            bool rest[SPL];
                            bool left = false, any = false;
#pragma unroll
                            for (int k = 0; k < SPL; ++k) {
                                const bool r = need[k] && !occl[k];
                                left = left || r;
                                rest[k] = r && (a.occ_mode != 1 || omesh[k] == mi);
                                any = any || rest[k];
                            }
                            if (ballot(left) == 0) break;
                            if (ballot(any) == 0) continue;
                            const BlasDesc b = a.blas[mi];
                            FixRec fo = fr;
                            float4 q[SPL];
#pragma unroll
                            for (int k = 0; k < SPL; ++k) q[k] = p[k];
                            if (moving) {
                                fo = load_fix(a.fix_all + (int64_t)mi * a.fix_stride, f);
                                if (mi != a.self_mesh) {
                                    const float* iv = a.xf + ((int64_t)mi * a.fix_stride + f) * 24 + 12;
#pragma unroll
                                    for (int k = 0; k < SPL; ++k) {
                                        const float wx = __builtin_fmaf(fw[0], p[k].x, __builtin_fmaf(fw[1], p[k].y, __builtin_fmaf(fw[2], p[k].z, fw[3])));
                                        const float wy = __builtin_fmaf(fw[4], p[k].x, __builtin_fmaf(fw[5], p[k].y, __builtin_fmaf(fw[6], p[k].z, fw[7])));
                                        const float wz = __builtin_fmaf(fw[8], p[k].x, __builtin_fmaf(fw[9], p[k].y, __builtin_fmaf(fw[10], p[k].z, fw[11])));
                                        q[k].x = __builtin_fmaf(iv[0], wx, __builtin_fmaf(iv[1], wy, __builtin_fmaf(iv[2], wz, iv[3])));
                                        q[k].y = __builtin_fmaf(iv[4], wx, __builtin_fmaf(iv[5], wy, __builtin_fmaf(iv[6], wz, iv[7])));
                                        q[k].z = __builtin_fmaf(iv[8], wx, __builtin_fmaf(iv[9], wy, __builtin_fmaf(iv[10], wz, iv[11])));
                                    }
                                }
                            }
                            bool o2[SPL];
                            packet_visibility<SPL>(a.blas_nodes + b.node_base, b.node_count, a.blas_tris + b.tri_base,
                                                   b.tri_count, fo.ex, fo.ey, fo.ez, fo.rx, fo.ry, fo.rz, q, otri, omesh,
                                                   2, rest, o2, n_visits);
#pragma unroll
                            for (int k = 0; k < SPL; ++k) occl[k] = occl[k] || o2[k];
                            ++n_trav;
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < SPL; ++k) {
                    const bool ok = g[k] > 0.0f && !occl[k];
                    n_vis += (uint32_t)__popcll(ballot(ok));
                    if (ok) s_acc[wave * (64 * SPL) + k * 64 + lane] += to_fixed(g[k], shift);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
        const int64_t i = wave_base + k * 64 + lane;
        const unsigned long long v = s_acc[wave * (64 * SPL) + k * 64 + lane];
        if (i < n && v != 0ull) atomicAdd(&a.acc[i], v);
    }
    if (lane == 0) {
        atomicAdd(&s_stats[0], n_in);
        atomicAdd(&s_stats[1], n_vis);
        atomicAdd(&s_stats[2], n_trav);
        atomicAdd(&s_stats[3], n_visits.nodes);
        atomicAdd(&s_stats[4], n_visits.tests);
        atomicAdd(&s_stats[5], n_bf);
    }
    __syncthreads();
    if (threadIdx.x < kDensityStats && s_stats[threadIdx.x]) atomicAdd(&a.stats[threadIdx.x], (unsigned long long)s_stats[threadIdx.x]);
    __syncthreads();  // LDS is reused by the next item of a persistent workgroup
}

// INST: visibility over one BVH per mesh (DensityLaunch::blas), else the scene BVH.
// Items in dispatch order go tile by tile, the chunks of one tile next to each other:
// workgroups are handed out round-robin over the XCDs, so the chunks of a tile run at
// once on different XCDs and every XCD sees every part of the scene; when only the
// first chunks hold fixations (a time window), the work still spreads over all XCDs.
// ZB: the paper's z-buffer visibility instead of the exact segment test.
// Occupancy: the one-sample-per-lane traversal kernels (this one, k_density_queue and
// k_zbuffer) ask for 8 waves per SIMD, the most the SIMD holds; their scalar registers
// then no longer fit and the compiler moves some long-lived ones (kernel arguments,
// mostly outside the walk) into vector-register lanes.  More waves hide more of the
// dependent node loads: the paper-shaped map takes 70.7 ms this way against 78.2 ms at
// the 7 waves the register counts allow otherwise.
template <int SPL, int OCC>
constexpr int kMinWaves = (SPL == 1 && OCC != 0) ? 8 : 1;

template <int SPL, int OCC, bool INST = false, bool ZB = false>
__global__ void __launch_bounds__(kThreads, (kMinWaves<SPL, OCC>)) k_density(DensityLaunch a)
{
    const unsigned L = blockIdx.x + blockIdx.y * gridDim.x;  // < 2^31 (tiles x chunks)
    const int F = a.F_live ? min(a.F, (int)*a.F_live) : a.F;
    density_item<SPL, OCC, kFB, INST, ZB>(a, (int64_t)(L / gridDim.y), (int)(L % gridDim.y), F);
}

// Persistent form for many sessions: every workgroup pulls (session, tile, chunk)
// items from a queue sorted longest first until the queue is empty.
template <int SPL, int FB>
__global__ void __launch_bounds__(kThreads, (SPL == 1 ? 8 : 1)) k_density_queue(const DensityLaunch* __restrict__ sessions,
                                                            const int4* __restrict__ items, int32_t n_items,
                                                            unsigned int* __restrict__ head)
{
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(head, 1u);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= n_items) break;
        const int4 w = items[it];
        // the session's descriptor stays in memory: its fields are read where they are
        // used (wave-uniform loads) rather than copied into registers
        density_item<SPL, 1, FB>(sessions[w.x], (int64_t)w.y, w.z, sessions[w.x].F);
    }
}

// ---------------------------------------------------------------------------
// a7: maximum and outputs in the caller's order
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_max(const unsigned long long* __restrict__ acc, int64_t n,
                                              unsigned long long* __restrict__ out)
{
    __shared__ unsigned long long s_m[4];
    unsigned long long m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, acc[i]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = max(m, (unsigned long long)__shfl_xor(m, d, 64));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = max(max(s_m[0], s_m[1]), max(s_m[2], s_m[3]));
        if (m) atomicMax(out, m);
    }
}

// In input order: each output is written where the caller expects it (coalesced), and
// gathers its accumulator from the point's sorted position.
__global__ void k_finalize(const unsigned long long* __restrict__ acc, const int32_t* __restrict__ inv, int64_t n,
                           const int32_t* __restrict__ shift_p, const unsigned long long* __restrict__ max_acc,
                           float* __restrict__ density, float* __restrict__ density_norm, float* __restrict__ max_out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int shift = *shift_p;
    const unsigned long long mx = *max_acc;
    if (j == 0 && max_out) *max_out = (float)ldexp((double)mx, -shift);
    if (j >= n) return;
    const unsigned long long v = acc[inv[j]];
    if (density) density[j] = (float)ldexp((double)v, -shift);
    if (density_norm) density_norm[j] = mx ? (float)((double)v / (double)mx) : 0.0f;
}

// ---------------------------------------------------------------------------
// stage-isolated checks
// ---------------------------------------------------------------------------
__global__ void k_pair_values(const float* __restrict__ pos, const FixRec* __restrict__ fix,
                              const int32_t* __restrict__ ps, const int32_t* __restrict__ pf, int64_t m,
                              int64_t n_points, int32_t F, float cone2, float kexp, float* __restrict__ g)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int64_t s = ps[i];
    const int32_t f = pf[i];
    if (s < 0 || s >= n_points || f < 0 || f >= F) {
        g[i] = __int_as_float(0x7fc00000);  // NaN marks an invalid pair
        return;
    }
    const FixRec fr = fix[f];
    g[i] = pair_value(pos[3 * s], pos[3 * s + 1], pos[3 * s + 2], fr.ex, fr.ey, fr.ez, fr.rx, fr.ry, fr.rz, fr.w,
                      cone2, kexp);
}

// one wave per pair, lane 0 active: the segment, its shear axis and its arithmetic
// are those the density kernel gives this pair (segment_axis of the fixation's gaze,
// or the segment's own dominant axis when `gaze` is NULL), and so is the back-face rule
// (bf.closed non-NULL); a pair's answer does not depend on the other segments of a
// packet.
__global__ void __launch_bounds__(64) k_pair_visibility(const float* __restrict__ pos, const int32_t* __restrict__ tri,
                                                        const int32_t* __restrict__ mesh,
                                                        const int32_t* __restrict__ tri_mesh,
                                                        const float* __restrict__ eye, const float* __restrict__ gaze,
                                                        const int32_t* __restrict__ ps,
                                                        const int32_t* __restrict__ pf, int64_t m, int64_t n_points,
                                                        int32_t n_eyes, int64_t T, const BvhNode* __restrict__ nodes,
                                                        const BvhTri* __restrict__ tris, int mode, BackfaceArgs bf,
                                                        uint8_t* __restrict__ vis)
{
    const int64_t i = blockIdx.x;
    if (i >= m) return;
    const int lane = lane_id();
    const int64_t s = ps[i];
    const int64_t f = pf[i];
    if (s < 0 || s >= n_points || f < 0 || f >= n_eyes) {
        if (lane == 0) vis[i] = 2;  // invalid pair
        return;
    }
    int t = tri ? tri[s] : -1;
    if (t < 0 || t >= T) t = -1;
    const int me = mesh ? mesh[s] : (t >= 0 ? tri_mesh[t] : -1);
    const float ex = eye[3 * f], ey = eye[3 * f + 1], ez = eye[3 * f + 2];
    const float px = pos[3 * s], py = pos[3 * s + 1], pz = pos[3 * s + 2];
    const float dx = px - ex, dy = py - ey, dz = pz - ez;
    const int kz = gaze ? segment_axis(dominant_axis(gaze[3 * f], gaze[3 * f + 1], gaze[3 * f + 2]), dx, dy, dz)
                        : dominant_axis(dx, dy, dz);
    int kx, ky;
    cyclic_axes(kz, kx, ky);
    const Seg sgs[1] = {make_seg(px, py, pz, ex, ey, ez, kx, ky, kz)};
    const float org[1][3] = {{px, py, pz}};
    TravCount visits;
    const int ot[1] = {t}, om[1] = {me};
    const bool act[1] = {mode != 0 && lane == 0};
    bool occ[1] = {false};
    const int oct = (signbit(dx) ? 1 : 0) | (signbit(dy) ? 2 : 0) | (signbit(dz) ? 4 : 0);
    if (bf.closed && mode != 0) {
        float nx, ny, nz;
        int cnt, cand[kBfCand];
        backface_point(px, py, pz, t, me, lane == 0, bf.V, bf.I, bf.closed, nodes, tris, bf.rmax, nx, ny, nz, cnt,
                       cand);
        if (lane == 0 && me >= 0 &&
            backface_rule(nx, ny, nz, cnt, [&cand](int j) { return cand[j]; }, px, py, pz, ex, ey, ez,
                          bf.mbox[2 * me], bf.mbox[2 * me + 1], bf.l2max, tris)) {
            vis[i] = 0;
            return;
        }
    }
    occluded_packet<1, false>(nodes, tris, org, oct, sgs, ot, om, mode, act, occ, visits);
    if (lane == 0) vis[i] = occ[0] ? 0 : 1;
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_fix_prep(const float* eye, const float* gaze, const float* dur, int32_t F, double sigma, double widen,
                     FixRec* rec, double* wsum, int32_t* fx_shift, hipStream_t s)
{
    (void)wsum;
    const double inv_norm = 1.0 / (sigma * std::sqrt(2.0 * M_PI));
    const double kappa_scale = (1.0 - widen) / (1.0 + 16.0 * sigma * sigma);
    unsigned int* wmax = reinterpret_cast<unsigned int*>(fx_shift + 1);
    if (F > 0) k_fix_prep<<<blocks(F, 256), 256, 0, s>>>(eye, gaze, dur, F, inv_norm, kappa_scale, rec, wmax);
    k_fix_shift<<<1, 1, 0, s>>>(wmax, F, fx_shift);
}

void launch_zcam_prep(const float* eye, const float* gaze, const float* dur, const float* head, int32_t F,
                      double sigma, double widen, double near_, double far_, FixRec* rec, ZCam* cam,
                      int32_t* fx_shift, hipStream_t s)
{
    const double inv_norm = 1.0 / (sigma * std::sqrt(2.0 * M_PI));
    unsigned int* wmax = reinterpret_cast<unsigned int*>(fx_shift + 1);
    if (F > 0)
        k_zcam_prep<<<blocks(F, 128), 128, 0, s>>>(eye, gaze, dur, head, F, sigma, inv_norm, widen, near_, far_, rec,
                                                   cam, wmax);
    k_fix_shift<<<1, 1, 0, s>>>(wmax, F, fx_shift);
}

void launch_zbuffer(const BvhNode* nodes, int64_t node_stride, const BvhTri* tris, int64_t tri_stride,
                    const FixRec* rec, const ZCam* cam, int32_t F, int32_t R, float* zbuf, hipStream_t s)
{
    const int64_t waves = (int64_t)F * (R / 8) * (R / 8);
    if (waves > 0) k_zbuffer<<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(nodes, node_stride, tris, tri_stride, rec, cam, F, R,
                                                                zbuf);
}

void launch_fix_posed(const float* eye, const float* gaze, const float* dur, const double* time, const float* pose,
                      int32_t F, int32_t M, int64_t stride, double t0, double t1, double sigma, double widen,
                      FixRec* rec, float* xf, unsigned int* kept, unsigned long long* budget,
                      unsigned long long* totals, hipStream_t s)
{
    const double inv_norm = 1.0 / (sigma * std::sqrt(2.0 * M_PI));
    const double kappa_scale = (1.0 - widen) / (1.0 + 16.0 * sigma * sigma);
    if (F > 0)
        k_fix_posed<<<blocks(F, 256), 256, 0, s>>>(eye, gaze, dur, time, pose, F, M, stride, t0, t1, inv_norm,
                                                   kappa_scale, rec, xf, kept, budget, totals);
}

void launch_fix_select(const float* eye, const float* gaze, const float* dur, const double* time, int32_t F,
                       double t0, double t1, double sigma, double widen, FixRec* rec, unsigned int* kept,
                       unsigned long long* budget, unsigned long long* totals, hipStream_t s)
{
    const double inv_norm = 1.0 / (sigma * std::sqrt(2.0 * M_PI));
    const double kappa_scale = (1.0 - widen) / (1.0 + 16.0 * sigma * sigma);
    if (F > 0)
        k_fix_select<<<blocks(F, 256), 256, 0, s>>>(eye, gaze, dur, time, F, t0, t1, inv_norm, kappa_scale, rec,
                                                    kept, budget, totals);
}

void launch_morton(const float* pos, const int32_t* tri, const int32_t* mesh, const int32_t* tri_mesh, int64_t n,
                   const float* bbox_lo, float inv_cell, int bits, uint32_t* key, uint32_t* hist, hipStream_t s)
{
    (void)tri; (void)mesh; (void)tri_mesh;
    if (n > 0)
        k_morton<<<blocks(n, 256), 256, 0, s>>>(pos, n, bbox_lo[0], bbox_lo[1], bbox_lo[2], inv_cell, 1 << bits, key,
                                                hist);
}

void launch_scatter(const float* pos, const int32_t* tri, const int32_t* mesh, const int32_t* tri_mesh, int64_t T,
                    int64_t n, const uint32_t* key, uint32_t* cursor, float4* spos, int32_t* smesh, int32_t* inv,
                    int32_t base, hipStream_t s)
{
    if (n > 0)
        k_scatter<<<blocks(n, 256), 256, 0, s>>>(pos, tri, mesh, tri_mesh, T, n, key, cursor, spos, smesh, inv,
                                                 base);
}

void launch_density(const DensityLaunch& a, hipStream_t s)
{
    if (a.n <= 0 || a.F <= 0) return;
    const int64_t per_tile = (int64_t)kThreads * a.spl;
    const dim3 grid(blocks(a.n, (int)per_tile), (unsigned)a.n_chunks);
    const bool occ = a.occ_mode != 0;
    if (a.zbuf) {
        if (a.spl == 1) k_density<1, 0, false, true><<<grid, kThreads, 0, s>>>(a);
        else k_density<2, 0, false, true><<<grid, kThreads, 0, s>>>(a);
        return;
    }
    if (occ && a.blas) {
        switch (a.spl) {
        case 1: k_density<1, 1, true><<<grid, kThreads, 0, s>>>(a); break;
        case 2: k_density<2, 1, true><<<grid, kThreads, 0, s>>>(a); break;
        default: k_density<4, 1, true><<<grid, kThreads, 0, s>>>(a); break;
        }
        return;
    }
    switch (a.spl) {
    case 1: occ ? k_density<1, 1><<<grid, kThreads, 0, s>>>(a) : k_density<1, 0><<<grid, kThreads, 0, s>>>(a); break;
    case 2: occ ? k_density<2, 1><<<grid, kThreads, 0, s>>>(a) : k_density<2, 0><<<grid, kThreads, 0, s>>>(a); break;
    default: occ ? k_density<4, 1><<<grid, kThreads, 0, s>>>(a) : k_density<4, 0><<<grid, kThreads, 0, s>>>(a); break;
    }
}

void launch_density_queue(const DensityLaunch* sessions, const int4* items, int32_t n_items, unsigned int* head,
                          int spl, int fb, int grid, hipStream_t s)
{
    if (n_items <= 0) return;
    const dim3 g((unsigned)grid);
#define GM_Q(S, B) k_density_queue<S, B><<<g, kThreads, 0, s>>>(sessions, items, n_items, head)
    if (fb <= 64) {
        if (spl == 1) GM_Q(1, 64); else if (spl == 2) GM_Q(2, 64); else GM_Q(4, 64);
    } else if (fb <= 128) {
        if (spl == 1) GM_Q(1, 128); else if (spl == 2) GM_Q(2, 128); else GM_Q(4, 128);
    } else {
        if (spl == 1) GM_Q(1, 256); else if (spl == 2) GM_Q(2, 256); else GM_Q(4, 256);
    }
#undef GM_Q
}

int density_queue_grid(int spl, int fb)
{
    int dev = 0, cus = 256, per = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipError_t e = hipSuccess;
#define GM_OCCQ(S, B) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_density_queue<S, B>, kThreads, 0)
    if (fb <= 64) {
        if (spl == 1) GM_OCCQ(1, 64); else if (spl == 2) GM_OCCQ(2, 64); else GM_OCCQ(4, 64);
    } else if (fb <= 128) {
        if (spl == 1) GM_OCCQ(1, 128); else if (spl == 2) GM_OCCQ(2, 128); else GM_OCCQ(4, 128);
    } else {
        if (spl == 1) GM_OCCQ(1, 256); else if (spl == 2) GM_OCCQ(2, 256); else GM_OCCQ(4, 256);
    }
#undef GM_OCCQ
    if (e != hipSuccess || per < 1) per = 1;
    return std::max(1, cus) * per;
}

void launch_finalize(const unsigned long long* acc, const int32_t* inv, int64_t n, const int32_t* fx_shift,
                     unsigned long long* max_acc, float* density, float* density_norm, float* max_out, hipStream_t s)
{
    if (n > 0) k_max<<<std::min<unsigned>(blocks(n, 256), 512u), 256, 0, s>>>(acc, n, max_acc);
    k_finalize<<<blocks(n > 0 ? n : 1, 256), 256, 0, s>>>(acc, inv, n, fx_shift, max_acc, density, density_norm,
                                                          max_out);
}

void launch_pair_values(const float* pos, const FixRec* fix, const int32_t* ps, const int32_t* pf, int64_t m,
                        int64_t n_points, int32_t F, float cone2, float kexp, float* g, hipStream_t s)
{
    if (m > 0) k_pair_values<<<blocks(m, 256), 256, 0, s>>>(pos, fix, ps, pf, m, n_points, F, cone2, kexp, g);
}

void launch_backface_prep(const float4* spos, const int32_t* smesh, int64_t n, const float* V, const int32_t* I,
                          const uint8_t* closed, const BvhNode* nodes, const BvhTri* tris, float rmax,
                          float4* bface, int32_t* bcand, hipStream_t s)
{
    if (n > 0) {
        const int lg = prep_lanes_log2(n);
        const int64_t waves = (n + (int64_t(1) << lg) - 1) >> lg;
        k_backface_prep<<<blocks(waves * 64, 256), 256, 0, s>>>(spos, smesh, n, V, I, closed, nodes, tris, rmax, lg,
                                                                bface, bcand);
    }
}

void launch_pair_visibility(const float* pos, const int32_t* tri, const int32_t* mesh, const int32_t* tri_mesh,
                            const float* eye, const float* gaze, const int32_t* ps, const int32_t* pf, int64_t m,
                            int64_t n_points, int32_t n_eyes, int64_t T, const BvhNode* nodes, const BvhTri* tris,
                            int32_t occ_mode, const BackfaceArgs& bf, uint8_t* vis, hipStream_t s)
{
    if (m > 0)
        k_pair_visibility<<<(unsigned)m, 64, 0, s>>>(pos, tri, mesh, tri_mesh, eye, gaze, ps, pf, m, n_points, n_eyes,
                                                     T, nodes, tris, occ_mode, bf, vis);
}

}  // namespace gm
