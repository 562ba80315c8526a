// gm_internal.h -- layouts and launchers shared by the host runtime and the
// gfx950 kernels of the density-map library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace gm {

// ---------------------------------------------------------------------------
// Occlusion BVH.  Two child boxes per node so that one 64-byte fetch feeds both
// box tests; nodes in depth-first order (the first child usually follows its
// parent); child >= 0 is a node index, child < 0 is a leaf whose triangles are
// tris[~child .. ~child + count).  An empty child has count 0 and an inverted box.
// ---------------------------------------------------------------------------
struct alignas(16) BvhNode {
    float lo0[3], hi0[3];
    float lo1[3], hi1[3];
    int32_t child0, child1;
    int32_t count0, count1;  // leaf triangle counts; count0 also carries the split axis
};
// count0 = leaf count | split axis << kSplitAxisShift: child 0 holds the triangles
// whose centroids lie lower along that axis.
constexpr int kSplitAxisShift = 8;
constexpr int kCountMask = (1 << kSplitAxisShift) - 1;
static_assert(sizeof(BvhNode) == 64, "node is one 64-byte line");

// Leaf triangle record, 48 bytes, in leaf order.
struct alignas(16) BvhTri {
    float v0[3], v1[3], v2[3];
    int32_t id;     // scene-global triangle index
    int32_t mesh;   // mesh of the triangle
    int32_t pad;
};
static_assert(sizeof(BvhTri) == 48, "triangle record is 48 bytes");

// Most triangles per leaf; the record array carries kLeafMax - 1 zeroed records past
// the end so a leaf's records can always be fetched as one group of kLeafMax.
constexpr int kLeafMax = 4;

// On the device the record array is stored three times, copy c holding the
// vertex coordinates in the axis order (kx, ky, kz) = ((c + 1) % 3, (c + 2) % 3, c),
// so that a wave whose segments share the dominant axis kz = c reads vertices
// already permuted for the watertight shear.  Copy 2 is the x, y, z order.
constexpr int kTriCopies = 3;
void permute_tri_copies(const std::vector<BvhTri>& in, std::vector<BvhTri>& out);

// The node array is stored eight times as well: in copy o, every axis a with bit a
// of o set has its box bounds swapped (lo holds the upper bound, hi the lower), so a
// wave whose segments all run towards -a along exactly those axes finds the near
// plane of each slab in lo and the far plane in hi.  Copy 0 is the plain array.
constexpr int kNodeCopies = 8;
void octant_node_copies(const std::vector<BvhNode>& in, std::vector<BvhNode>& out);

// Per-fixation record written by the prep kernel (32 bytes).
struct alignas(16) FixRec {
    float ex, ey, ez;  // eye
    float rx, ry, rz;  // gaze, as given (not normalised)
    float w;           // t / (sigma sqrt(2 pi))
    float kappa;       // |r|^2 / (1 + 16 sigma^2), widened: the cheap cone gate's factor
};

// Host-side BVH (bvh_build.cpp).
struct HostBvh {
    std::vector<BvhNode> nodes;
    std::vector<BvhTri> tris;
    int depth = 0;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
};
// leaf_max (1 .. kLeafMax): most triangles per leaf.
void build_bvh(const float* V, const int32_t* I, const int32_t* tri_mesh, int64_t T, HostBvh& out,
               int leaf_max = kLeafMax);

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files).  All asynchronous on `s`.
// ---------------------------------------------------------------------------

// a1: areas and per-mesh max (max_bits: uint64 [M], zeroed by the caller).
// y[i] = sqrt(x[i]) in FP64 with the sampler's code generation (a diagnostic of its rounding).
void launch_sqrt_f64(const double* x, double* y, int64_t n, hipStream_t s);
void launch_tri_area(const float* V, const int32_t* I, const int32_t* tri_mesh, int64_t T, double* area,
                     unsigned long long* max_bits, hipStream_t s);
// a1: per-mesh scale exponent S_m from T_m and the max area.
void launch_mesh_scale(const unsigned long long* max_bits, const int64_t* tri_off, int32_t M, int32_t* S,
                       hipStream_t s);
// a1: fixed-point weights W_i = floor(A_i 2^S_m).
void launch_tri_weight(const double* area, const int32_t* tri_mesh, const int32_t* S, int64_t T,
                       unsigned long long* W, hipStream_t s);
// Lattice sampler: per-triangle point counts from the areas, per-mesh totals from
// their inclusive scan C, and the points themselves.
void launch_lattice_count(const double* area, int64_t T, double k, unsigned long long* cnt, hipStream_t s);
void launch_lattice_mesh_counts(const unsigned long long* C, const int64_t* tri_off, int32_t M, int64_t* counts,
                                hipStream_t s);
void launch_lattice_sample(const float* V, const int32_t* I, const int32_t* tri_mesh, const double* area,
                           const unsigned long long* C, int64_t T, int64_t N, double k, int32_t* tri, int32_t* mesh,
                           float* bary, float* pos, hipStream_t s);

// a2: inclusive prefix sum of uint64 over n (tmp: scan_tmp_bytes(n)).
size_t scan_tmp_bytes(int64_t n);
void launch_inclusive_scan_u64(const unsigned long long* in, unsigned long long* out, int64_t n, void* tmp,
                               hipStream_t s);
void launch_exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* tmp, hipStream_t s);
// a2: per-mesh totals and sample counts/offsets: counts [M], offsets [M+1] (int64).
void launch_mesh_counts(const unsigned long long* C, const int64_t* tri_off, const int32_t* S, int32_t M,
                        double k, int64_t* counts, int64_t* offsets, unsigned long long* mesh_total,
                        hipStream_t s);
// a3: the sampler.
void launch_sample(const float* V, const int32_t* I, const unsigned long long* C, const int64_t* tri_off,
                   const int64_t* offsets, const unsigned long long* mesh_total, const int32_t* guide,
                   const int64_t* goff, const int32_t* gsh, int32_t M, int64_t N, uint64_t seed, int32_t* tri,
                   int32_t* mesh, float* bary, float* pos, hipStream_t s);
// guide[goff[m] + k] for k <= (mesh_total[m] - 1) >> gsh[m]: the first triangle t of mesh m
// with C[t] > C[start of m] + (k << gsh[m]); the entry after the last bucket holds the mesh's
// last triangle (G entries in all)
void launch_sample_guide(const unsigned long long* C, const int64_t* tri_off, const int64_t* goff,
                         const int32_t* gsh, int32_t M, int64_t G, int32_t* guide, hipStream_t s);

// density path
// in-cone pairs, visible pairs, packet traversals, BVH node visits, triangle tests (wave level),
// pairs settled by the back-face rule, (work item, fixation) pairs kept by the tile cone test
constexpr int kDensityStats = 7;
// Tolerance of the exact visibility test (the exact counterpart of the depth test of
// Sec. 3.2.2): a hit occludes when its parameter tau on the segment eye + tau (x - eye)
// lies in (0, 1 - kEpsV).  The kernels take the bound as a compile-time constant.
constexpr double kEpsV = 1e-4;
// One mesh's BVH inside the concatenated per-mesh arrays: kNodeCopies copies of
// node_count nodes from node_base, kTriCopies copies of tri_count records from tri_base.
struct BlasDesc {
    int64_t node_base, node_count, tri_base, tri_count;
};

struct DensityLaunch {
    // sorted samples
    const float4* spos;        // xyz, w = own triangle (int bits, -1 = none)
    const int32_t* smesh;      // own mesh (-1 = none)
    int64_t n;
    const FixRec* fix;
    int32_t F;
    const BvhNode* nodes;      // kNodeCopies octant copies
    int64_t node_stride;       // nodes per copy
    const BvhTri* tris;        // kTriCopies permuted copies
    int64_t tri_stride;        // records per copy
    int32_t occ_mode;
    float cone2;               // 16 sigma^2
    float kexp;                // log2(e) / (2 sigma^2)
    const int32_t* fx_shift;   // device scalar: fixed-point scale exponent
    unsigned long long* acc;   // [n] fixed-point density, sorted order
    unsigned long long* stats; // [kDensityStats] counters of the call
    int32_t fix_per_chunk;
    int32_t n_chunks;
    int32_t spl;               // samples per lane
    const unsigned int* F_live = nullptr;  // device count of valid records (<= F), or NULL: all F
    // One BVH per mesh (blas, n_inst of them; NULL: the scene BVH above).  Static
    // scenes: xf and fix_all NULL, every mesh in the world frame.  Posed launches
    // (meshes that move between fixations, one launch per mesh self_mesh): fixation
    // records per mesh (fix = fix_all + self_mesh * fix_stride) and per (mesh,
    // fixation) 24 floats, the 3x4 pose (mesh -> world) and then its inverse.
    const BlasDesc* blas = nullptr;
    const BvhNode* blas_nodes = nullptr;
    const BvhTri* blas_tris = nullptr;
    const FixRec* fix_all = nullptr;
    const float* xf = nullptr;
    int64_t fix_stride = 0;
    int32_t n_inst = 0;
    int32_t self_mesh = 0;
    // The paper's z-buffer visibility (zbuf != NULL): per fixation a camera record
    // (ZCam, 16 floats) and a zres x zres buffer of nearest depths; a pair counts
    // when the point lies in the cropped frustum and its depth D has D - zbuf <= zeps D.
    const float* zcam = nullptr;
    const float* zbuf = nullptr;
    int32_t zres = 0;
    float zeps = 0.0f;
    // The back-face rule (static scenes; NULL bface: off).  Per sorted point: the unit
    // normal of its own triangle times the point's distance to that triangle's edges
    // and, in w, the number of triangles of its mesh within
    // bf_rmax of it (as int bits; -1: the rule does not apply to the point), whose
    // record indices (plain x, y, z copy) are bcand[kBfCand * i + j].  mbox: per mesh the
    // bounding box, lo then hi (2 float4).  A segment longer than sqrt(bf_L2max) is left
    // to the traversal.
    const float4* bface = nullptr;
    const int32_t* bcand = nullptr;
    const float4* mbox = nullptr;
    const BvhTri* bf_tris = nullptr;
    float bf_L2max = 0.0f;
};

// Triangles of its own mesh listed per point for the back-face rule (more: the rule
// does not apply to the point).
constexpr int kBfCand = 8;

// Camera of one fixation for the z-buffer test: right, up, forward unit vectors, the
// crop's NDC scale and offset (x_ndc = sx x / D - ox, y likewise, D the depth along
// forward), the near and far depths.
struct alignas(16) ZCam {
    float x[3], y[3], f[3];
    float sx, ox, sy, oy;
    float near_, far_;
    float pad;
};
static_assert(sizeof(ZCam) == 64, "camera record is 64 bytes");


void launch_fix_prep(const float* eye, const float* gaze, const float* dur, int32_t F, double sigma,
                     double widen, FixRec* rec, double* wsum, int32_t* fx_shift, hipStream_t s);
// z-buffer visibility: per fixation the camera, its crop to the 4-sigma cone (Appendix A)
// and a gate record whose cone holds the crop (rec.w = 0 for a fixation whose crop is
// undefined); then one nearest-depth ray per pixel centre
void launch_zcam_prep(const float* eye, const float* gaze, const float* dur, const float* head, int32_t F,
                      double sigma, double widen, double near_, double far_, FixRec* rec, ZCam* cam,
                      int32_t* fx_shift, hipStream_t s);
// nodes: kNodeCopies octant copies node_stride apart; tris: kTriCopies axis copies tri_stride apart
void launch_zbuffer(const BvhNode* nodes, int64_t node_stride, const BvhTri* tris, int64_t tri_stride,
                    const FixRec* rec, const ZCam* cam, int32_t F, int32_t R, float* zbuf, hipStream_t s);
// posed maps: per fixation taken, one record and one pose pair (forward, inverse) per mesh
void launch_fix_posed(const float* eye, const float* gaze, const float* dur, const double* time, const float* pose,
                      int32_t F, int32_t M, int64_t stride, double t0, double t1, double sigma, double widen,
                      FixRec* rec, float* xf, unsigned int* kept, unsigned long long* budget,
                      unsigned long long* totals, hipStream_t s);
// incremental maps: records of the fixations of one block that fall in a time window
void launch_fix_select(const float* eye, const float* gaze, const float* dur, const double* time, int32_t F,
                       double t0, double t1, double sigma, double widen, FixRec* rec, unsigned int* kept,
                       unsigned long long* budget, unsigned long long* totals, hipStream_t s);
void launch_morton(const float* pos, const int32_t* tri, const int32_t* mesh, const int32_t* tri_mesh,
                   int64_t n, const float* bbox_lo, float inv_cell, int bits, uint32_t* key, uint32_t* hist,
                   hipStream_t s);
void launch_scatter(const float* pos, const int32_t* tri, const int32_t* mesh, const int32_t* tri_mesh,
                    int64_t T, int64_t n, const uint32_t* key, uint32_t* cursor, float4* spos, int32_t* smesh,
                    int32_t* inv, int32_t base, hipStream_t s);  // inv[i] = base + sorted position of point i
void launch_density(const DensityLaunch& a, hipStream_t s);
// persistent multi-session form: items are (session, tile, chunk, 0); head is zeroed by the caller
void launch_density_queue(const DensityLaunch* sessions, const int4* items, int32_t n_items, unsigned int* head,
                          int spl, int fb, int grid, hipStream_t s);
// persistent workgroups that fit on the device at once for that kernel
int density_queue_grid(int spl, int fb);
void launch_finalize(const unsigned long long* acc, const int32_t* inv, int64_t n, const int32_t* fx_shift,
                     unsigned long long* max_acc, float* density, float* density_norm, float* max_out,
                     hipStream_t s);
void launch_pair_values(const float* pos, const FixRec* fix, const int32_t* ps, const int32_t* pf, int64_t m,
                        int64_t n_points, int32_t F, float cone2, float kexp, float* g, hipStream_t s);
// The scene's back-face rule data for gm_debug_pair_visibility (closed NULL: no rule).
struct BackfaceArgs {
    const float* V = nullptr;
    const int32_t* I = nullptr;
    const uint8_t* closed = nullptr;
    const float4* mbox = nullptr;
    float rmax = 0.0f;
    float l2max = 0.0f;
};
void launch_pair_visibility(const float* pos, const int32_t* tri, const int32_t* mesh, const int32_t* tri_mesh,
                            const float* eye, const float* gaze, const int32_t* ps, const int32_t* pf, int64_t m,
                            int64_t n_points, int32_t n_eyes, int64_t T, const BvhNode* nodes, const BvhTri* tris,
                            int32_t occ_mode, const BackfaceArgs& bf, uint8_t* vis, hipStream_t s);

// ---------------------------------------------------------------------------
// Neural density field: 96 Fourier features -> 4 x (64, ReLU) -> 1 -> softplus.
// Master parameters are FP32 in one flat array:
//   W1 [96][64] (input, output), b1 [64], W2 [64][64], b2, W3, b3, W4, b4, w5 [64], b5.
// ---------------------------------------------------------------------------
constexpr int kFieldBands = 16;
constexpr int kFieldFeat = 6 * kFieldBands;
constexpr int kFieldWidth = 64;
constexpr int kFieldOffW[5] = {0, 0, 6208, 10368, 14528};   // W_L, L = 1..4
constexpr int kFieldOffB[5] = {0, 6144, 10304, 14464, 18624};  // b_L
constexpr int kFieldOffW5 = 18688;
constexpr int kFieldOffB5 = 18752;
constexpr int kFieldParams = 18753;
size_t field_pack_bytes();   // bf16 image of the parameters in matrix-core operand order
size_t field_infer_bytes();  // its prefix used by inference

struct FieldGeom {
    float lo[3];
    float inv_ext;
    float freq[kFieldBands];
};

struct FieldTrain {
    const float* pos;        // [n][3]
    const float* target;     // [n]
    const int32_t* idx;      // training subset (NULL: the first `batch` points in order)
    int64_t n_idx;
    int32_t batch;           // points of this step
    float inv_batch;         // 1 / batch
    uint32_t key0, key1;     // Philox key of the batch draw
    uint32_t step;
    float* gpart;            // [slots][kFieldParams] per-wave gradient sums (per network)
    double* lpart;           // [slots] per-wave sums of squared errors (per network)
    int32_t slots;           // set by the launchers: field_train_slots(batch, networks)
};

// Several networks in one launch (blockIdx.y = network): geometry, and the start and
// number of each network's training indices in FieldTrain::idx (0: nothing to train),
// packed images pack_stride bytes apart.  off == NULL: one network, as passed.
struct FieldNets {
    const FieldGeom* geom = nullptr;
    const int64_t* off = nullptr;
    const int64_t* cnt = nullptr;
    int64_t pack_stride = 0;
};

void launch_field_pack(const float* master, unsigned char* blob, hipStream_t s);
// the packed images of M networks (parameters kFieldParams apart, images field_pack_bytes() apart)
void launch_field_pack_nets(const float* master, unsigned char* blob, int32_t M, hipStream_t s);
// Points whose mesh (mesh[i], else tri_mesh[tri[i]] for 0 <= tri[i] < T) is `m` get the
// network's value; m < 0 writes every point.
struct FieldRoute {
    const int32_t* mesh;
    const int32_t* tri;
    const int32_t* tri_mesh;
    int64_t T;
    int32_t m;
};
void launch_field_infer(const unsigned char* blob, const FieldGeom& g, const float* pos, int64_t q, float* out,
                        const FieldRoute& route, hipStream_t s);
// All networks in one launch, each over its own mesh's points only (route: the points'
// meshes; take[m] != 0 selects the routed meshes, NULL: all).  Scratch: cnt [3 M], base
// [3 M + 1], ridx [field_route_slots(q, M)], and per-chunk counts part
// [field_route_part_bytes(q, M) bytes] (0 bytes: pass NULL, the counts then go through
// global atomics).  A mesh whose points are contiguous in the input is read in place (no
// list entries).
int64_t field_route_slots(int64_t q, int32_t M);
int64_t field_route_part_bytes(int64_t q, int32_t M);
void launch_field_infer_routed(const unsigned char* blobs, int64_t pack_stride, const FieldGeom* geoms,
                               const float* pos, int64_t q, float* out, const FieldRoute& route,
                               const uint8_t* take, int32_t M, unsigned int* cnt, unsigned int* part, int64_t* base,
                               int32_t* ridx, hipStream_t s);
// sel[i] = flag[i] && mesh[i] == m
void launch_field_select(const uint32_t* flag, const int32_t* mesh, int32_t m, int64_t n, uint32_t* sel, hipStream_t s);
// One training step's forward and backward pass: the gradient grad [kFieldParams] and the
// sum of squared errors loss [1], reduced in a fixed order from the per-wave slots
// t.gpart / t.lpart (field_train_slots(batch, 1) of them).
int32_t field_train_slots(int32_t batch, int32_t M);
void launch_field_train(const unsigned char* blob, const FieldGeom& g, FieldTrain t, float* grad, double* loss,
                        hipStream_t s);
// the same for M networks at once (see FieldNets; t.key0 is xored with the network):
// grad [M][kFieldParams], loss [M], slots field_train_slots(batch, M) per network
void launch_field_train_nets(const unsigned char* blob, const FieldNets& nets, int32_t M, FieldTrain t, float* grad,
                             double* loss, hipStream_t s);
void launch_field_adam(float* master, float* m, float* v, float* grad, int64_t count, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);
// held-out split and per-mesh error sums
void launch_field_split(int64_t n, uint32_t key0, uint32_t key1, uint32_t threshold, uint32_t* flag_train,
                        hipStream_t s);
void launch_field_compact(const uint32_t* flag, const uint32_t* offs, int64_t n, int32_t* idx, hipStream_t s);
// sums[2 m], sums[2 m + 1]: squared error and squared target over the held-out points of
// mesh m, summed in a fixed order; part: field_l2_part_bytes(n, M) bytes of scratch
int64_t field_l2_part_bytes(int64_t n, int32_t M);
void launch_field_l2(const float* pred, const float* target, const int32_t* mesh, const uint32_t* flag_train,
                     int64_t n, int32_t M, double* part, double* sums, hipStream_t s);
// query helpers
void launch_gate_flags(const int32_t* mesh, const int32_t* tri, const int32_t* tri_mesh, int64_t T,
                       const uint8_t* gate, int32_t M, int64_t q, uint32_t* need, hipStream_t s);
void launch_gather_points(const float* pos, const int32_t* tri, const int32_t* mesh, const uint32_t* need,
                          const uint32_t* offs, int64_t q, float* gpos, int32_t* gtri, int32_t* gmesh, int32_t* gidx,
                          hipStream_t s);
void launch_scatter_fallback(const float* rho, const int32_t* gidx, int64_t m, const float* norm, float* out,
                             hipStream_t s);
void launch_used_flags(const uint32_t* need, int64_t q, uint8_t* used, hipStream_t s);

// true when the mesh bounds a solid: closed, consistently wound, outward (host)
bool mesh_is_closed(const float* V, int64_t nv, const int32_t* I, int64_t T);
// Per sorted point, the data of the back-face rule (see DensityLaunch::bface): normal of
// its own triangle and the triangles of its mesh whose boxes come within rmax of it,
// found by a packet walk of the scene BVH (plain node copy `nodes`, record copy `tris`
// in x, y, z order).  closed [M] (device): meshes the rule may use.
void launch_backface_prep(const float4* spos, const int32_t* smesh, int64_t n, const float* V, const int32_t* I,
                          const uint8_t* closed, const BvhNode* nodes, const BvhTri* tris, float rmax,
                          float4* bface, int32_t* bcand, hipStream_t s);

}  // namespace gm
