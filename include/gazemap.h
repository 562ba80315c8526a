/*
 * gazemap.h -- C ABI of the MI355X (gfx950) surface-based fixation density map library.
 *
 * The method (Javerliat & Lavoue, "GPU accelerated surface-based gaze mapping
 * for XR experiences", arXiv 2601.07571):
 *   1. sample every mesh surface at k samples per square metre, independently of
 *      the triangulation and of any UV mapping (Sec. 3.1);
 *   2. for every sample, add the duration-weighted angular Gaussian of every
 *      fixation whose 4-sigma gaze cone contains it and that sees it
 *      (Sec. 3.2.1, Sec. 3.2.2, Sec. 3.3.2);
 *   3. divide by the largest value (Sec. 3.2.3).
 *
 * Conventions shared by every call
 *   - Return value: GM_OK or a negative gm_status; gm_last_error() then holds a
 *     message (thread-local, valid until the next call on the same thread).
 *     Nothing is thrown across the ABI.  On error no output is written, unless
 *     the status is GM_ERR_DEVICE (a kernel may already have run).
 *   - Device pointers are HIP device allocations owned by the caller (for
 *     example torch tensors).  Host pointers are marked "host".
 *   - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *     Calls are asynchronous on that stream unless documented as blocking.
 *   - Positions are world-space metres, float32, laid out [n][3].
 *   - Scene-global triangle index: triangles of mesh 0 first, then mesh 1, ...
 *   - Handles (gm_scene) are not thread-safe: one call at a time per handle.
 */
#ifndef GAZEMAP_H
#define GAZEMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GM_OK = 0,
    GM_ERR_INVALID_ARGUMENT = -1,
    GM_ERR_OUT_OF_MEMORY = -2,
    GM_ERR_DEVICE = -3,
    GM_ERR_CAPACITY = -4,
    GM_ERR_NOT_READY = -5,
    GM_ERR_INTERNAL = -99
} gm_status;

/* Occlusion modes (Sec. 3.2.2), low two bits of `flags`. */
#define GM_OCC_NONE 0u  /* every in-cone sample counts */
#define GM_OCC_SELF 1u  /* only triangles of the sample's own mesh occlude */
#define GM_OCC_FULL 2u  /* every triangle of the scene occludes */
#define GM_OCC_MASK 3u

/* Thread-local message of the last failing call ("" if none). */
const char* gm_last_error(void);

/* ABI version, (major << 16) | minor. */
int32_t gm_version(void);

/* One triangle mesh, host memory: vertices [n_vertices][3] float32,
 * indices [n_triangles][3] int32 into this mesh's own vertices. */
typedef struct {
    const float* vertices;
    const int32_t* indices;
    int32_t n_vertices;
    int32_t n_triangles;
} gm_mesh;

typedef struct gm_scene gm_scene;

/*
 * gm_scene_create -- copy meshes to the current HIP device and build the
 * occlusion BVH on the host (binned SAH over triangle centroids, two child
 * boxes per 64-byte node in depth-first order, 48-byte triangle records in
 * leaf order).  Blocking.  Rejects: n_meshes < 1 or > 4096, a mesh with no
 * triangles, an index outside its mesh, a non-finite vertex.  Degenerate
 * (zero-area) triangles are accepted: they are never sampled and never occlude.
 * Three environment variables, read here, override tuning choices for measurement
 * (results are bit-identical under each; invalid values are ignored):
 *   GM_BVH_LEAF          most triangles per BVH leaf, 1..4 (default 4);
 *   GM_SAMPLES_PER_LANE  sample slots per lane of the density kernels, 1, 2 or 4
 *                        (default 1 with a visibility test, 2 without);
 *   GM_FIX_PER_CHUNK     fixations per work item of a density launch, > 0
 *                        (default: chosen per launch from the tile and fixation counts).
 */
gm_status gm_scene_create(const gm_mesh* meshes, int32_t n_meshes, gm_scene** out);
gm_status gm_scene_destroy(gm_scene* scene);

/* Host outputs (any may be NULL): triangle count, mesh count, BVH node count,
 * BVH depth, scene bounding box [6] = (lo xyz, hi xyz). */
gm_status gm_scene_info(const gm_scene* scene, int64_t* n_triangles, int32_t* n_meshes,
                        int64_t* n_bvh_nodes, int32_t* bvh_depth, float* bbox);

/*
 * gm_scene_mesh_closed -- host uint8 closed [n_meshes]: 1 for the meshes the visibility
 * test treats as bounding a solid (gm_mesh_closed at creation, unless cleared).  For such
 * a mesh a point seen from behind (the eye on the inner side of its triangle's plane, with
 * c D >= 4 eta: c the cosine between the segment and the plane's normal, D the point's
 * distance to its triangle's edges, eta = 2^-24 (|x| + |y| + |z|) the FP32 spacing at the
 * point), from an eye outside the mesh's bounding box, is occluded by
 * the mesh itself (Sec. 3.2.2's visibility: the segment must enter the solid before it
 * reaches the point); accumulate_density then skips the BVH walk for the pair when no
 * triangle of the mesh other than the point's own comes within 1e-4 of the segment's
 * length of the point (so the entry lies before the tolerance), and walks otherwise
 * (also for segments longer than twice the scene's diagonal plus 4 m).
 * gm_scene_set_mesh_closed -- clear (closed = 0) or restore (1; only for a mesh that
 * passed gm_mesh_closed) the flag of one mesh, e.g. for a closed mesh that intersects
 * itself with inverted parts.  Blocking (synchronises the device).
 */
gm_status gm_scene_mesh_closed(const gm_scene* scene, uint8_t* closed);
gm_status gm_scene_set_mesh_closed(gm_scene* scene, int32_t mesh, int32_t closed);

/*
 * gm_mesh_closed -- whether a mesh (host arrays, as gm_mesh) bounds a solid: after
 * merging vertices at identical positions, every directed edge of its triangles occurs
 * once and its reverse once (closed, edge-manifold, consistently wound), no triangle
 * repeats a vertex, and its signed volume is positive (normals (v1 - v0) x (v2 - v0)
 * point outwards).  Self-intersection is not checked.  Returns 1 or 0, -1 for invalid
 * arguments.  Host only (no device).  gm_scene_create applies it to every mesh; the
 * visibility test uses it for the back-face rule (a sample seen from behind on a
 * closed mesh, from an eye outside the mesh's box, is occluded by that mesh: Sec. 3.2.2).
 */
int32_t gm_mesh_closed(const float* vertices, int32_t n_vertices, const int32_t* indices, int32_t n_triangles);

/*
 * gm_count_surface_samples -- per-mesh sample counts for `samples_per_m2` (Sec. 3.1.2:
 * the count follows the surface area): n_m = round(k * area_m), where area_m is
 * the mesh area held as fixed-point triangle weights (floor(A_i * 2^S_m),
 * S_m = 52 - exponent(T_m * max_i A_i)).  n_per_mesh: host int64 [n_meshes].
 * The weights do not depend on the density: the first sampling call on a scene
 * computes them on the device and reads the per-mesh totals back (blocking, once);
 * afterwards the counts are evaluated on the host and this call does no device work.
 * samples_per_m2 must be finite and > 0.
 */
gm_status gm_count_surface_samples(gm_scene* scene, double samples_per_m2, int64_t* n_per_mesh,
                                   void* stream);

/*
 * build_surface_samples -- area-weighted surface sampling (Sec. 3.1; the
 * per-triangle lattice of Sec. 3.1.1 is replaced by area-proportional random
 * placement, so the density does not depend on the triangulation).
 *   a1  per-triangle FP64 area, fixed-point weight;
 *   a2  exact integer prefix sum of the weights (per mesh);
 *   a3  sample j of mesh m: Philox4x32-10(counter = (j_lo, j_hi, m, 0),
 *       key = (seed_lo, seed_hi)) -> triangle = first i with C_i > floor(U*W_m/2^64),
 *       U = x0*2^32 + x1; barycentric (1-sqrt(u), sqrt(u)(1-v), sqrt(u) v),
 *       u = x2/2^32, v = x3/2^32; position in FP64, rounded to FP32.
 * Sample order: mesh 0 first, then by j.  Outputs (device, caller-owned, each may
 * be NULL): tri [N] scene-global triangle index, mesh [N], bary [N][2] = (b1, b2),
 * pos [N][3].  N = sum of gm_count_surface_samples; N > capacity gives
 * GM_ERR_CAPACITY with *n_out = N and nothing written.  *n_out (host) = N.
 * Queued on `stream` (the per-mesh counts come from the scene's weight totals kept on
 * the host); only the first sampling call on a scene blocks, once, while a1 and a2
 * run and their totals are read back.  The scene's count buffers are rewritten by
 * each call: calls on one scene queued on different streams race unless the caller
 * synchronises them.
 */
gm_status build_surface_samples(gm_scene* scene, double samples_per_m2, uint64_t seed,
                                int32_t* tri, int32_t* mesh, float* bary, float* pos,
                                int64_t capacity, int64_t* n_out, void* stream);

/*
 * gm_count_lattice_samples -- per-mesh point counts of the paper's own sampler
 * (Sec. 3.1.1, 3.1.2): triangle i of area A_i (the same FP64 area as above) is
 * subdivided at resolution r_i = 1 if Delta_i = 8 k A_i + 1 < 25, else
 * floor((sqrt(Delta_i) - 3) / 2) (Eq. 4, the real root truncated to a whole
 * resolution), and holds (r_i + 1)(r_i + 2) / 2 points (Eq. 1).  n_per_mesh: host
 * int64 [n_meshes].  Blocking.  samples_per_m2 must be in (0, 1e12].
 */
gm_status gm_count_lattice_samples(gm_scene* scene, double samples_per_m2, int64_t* n_per_mesh, void* stream);

/*
 * build_lattice_samples -- every lattice point of the scene, in mesh order, then
 * triangle order, then index idx within the triangle.  Eq. (2): row =
 * ceil((sqrt(8 idx + 9) - 3) / 2), made exact with integers (f(row - 1) <= idx <
 * f(row)), col = idx - f(row - 1).  Eq. (3) as printed does not sum to one; it is
 * completed to w1 = col / r, w2 = (r - row) / r, w3 = (row - col) / r, which
 * enumerates the lattice {(i, j, l) / r : i + j + l = r}; P = w1 v0 + w2 v1 + w3 v2
 * in FP64, rounded to FP32.  Outputs as for build_surface_samples (device,
 * caller-owned, each may be NULL): tri [N] scene-global, mesh [N], bary [N][2] =
 * (w2, w3), pos [N][3].  N > capacity gives GM_ERR_CAPACITY with *n_out = N and
 * nothing written.  Blocking (it reads back the counts).
 */
gm_status build_lattice_samples(gm_scene* scene, double samples_per_m2, int32_t* tri, int32_t* mesh, float* bary,
                                float* pos, int64_t capacity, int64_t* n_out, void* stream);

/* Fixations, device memory: eye [n][3] and gaze [n][3] (direction, any non-zero
 * length) in world space, duration [n] >= 0 (the weight t of Sec. 3.2.1). */
typedef struct {
    const float* eye;
    const float* gaze;
    const float* duration;
    int32_t n;
} gm_fixations;

/*
 * accumulate_density -- the density map of Sec. 3.2 on a set of surface points.
 * For every point s and fixation f, with p = x_s - e_f and r_f the gaze:
 *   tan(phi) = |p x r| / (p . r), sigma = tan(theta);
 *   in the cone  <=>  p . r > 0 and tan(phi) <= 4 sigma          (Sec. 3.3.2);
 *   g = t_f / (sigma sqrt(2 pi)) * exp(-tan^2(phi) / (2 sigma^2))  (Sec. 3.2.1,
 *       sigma_k = (d2/d) sigma = tan(phi));
 *   visible  <=>  no occluding triangle other than tri[s] crosses the segment
 *       e_f + tau (x_s - e_f) at 0 < tau < 1 - 1e-4               (Sec. 3.2.2);
 *   rho_s = sum over in-cone visible f of g.
 * Inputs (device): pos [n][3]; tri [n] scene-global triangle of each point or NULL
 * (no own-triangle exclusion); mesh [n] or NULL (then derived from tri; points
 * with neither have no own mesh, so GM_OCC_SELF gives them no occluders).
 * flags: one GM_OCC_* mode.  theta_deg in (0, 45).
 * Outputs (device, each may be NULL): density [n] = rho (float32);
 * density_norm [n] = rho / max rho (Sec. 3.2.3; all zero when max is 0);
 * max_out [1] = max rho.
 * Accumulation is exact integer fixed point, so results do not depend on the
 * order of work (bit-reproducible).  Queued on `stream`; device scratch is held
 * by the scene handle and grown on demand (the first call for a size allocates).
 */
gm_status accumulate_density(gm_scene* scene, const float* pos, const int32_t* tri,
                             const int32_t* mesh, int64_t n, const gm_fixations* fix,
                             double theta_deg, uint32_t flags, float* density,
                             float* density_norm, float* max_out, void* stream);

/*
 * accumulate_density_noalloc -- accumulate_density for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, kernels and results (bit for bit) as
 * accumulate_density; its intermediate buffers live in one fixed device array of
 * gm_noalloc_scratch_bytes() bytes per device, held until the process ends, so it
 * calls no device allocation.  Limits: n <= GM_NOALLOC_MAX_POINTS points and
 * fix->n <= GM_NOALLOC_MAX_FIXATIONS fixations, else GM_ERR_CAPACITY with nothing
 * queued.  All calls on one device share that array: calls that overlap on one
 * device (different streams or threads) race; serialise them.  Queued on `stream`.
 */
#define GM_NOALLOC_MAX_POINTS 524288
#define GM_NOALLOC_MAX_FIXATIONS 65536
gm_status accumulate_density_noalloc(gm_scene* scene, const float* pos, const int32_t* tri,
                                     const int32_t* mesh, int64_t n, const gm_fixations* fix,
                                     double theta_deg, uint32_t flags, float* density,
                                     float* density_norm, float* max_out, void* stream);
int64_t gm_noalloc_scratch_bytes(void);

/*
 * Stage-isolated checks (same device code as accumulate_density), for tests.
 * gm_debug_pair_values: for m pairs (pair_s[i], pair_f[i]) (device int32) of the
 *   n_points points pos [n_points][3] and the fixations, g_out[i] (device float) = g
 *   (Sec. 3.2.1) if the pair is in the 4-sigma cone, else 0; no visibility.  A pair
 *   index out of range gives NaN.  Blocking (it owns a temporary buffer).
 * gm_debug_sqrt_f64: y[i] = sqrt(x[i]) for n device doubles, by the FP64 square
 *   root as the sampler's code evaluates it (the canonical triangle area of Sec. 3.1
 *   and the square-root warp of the placement both take it); bit-exact sample
 *   positions need it correctly rounded, which this lets a test check.  Queued on
 *   `stream`; x and y may be the same buffer.
 * gm_debug_pair_visibility: vis_out[i] (device uint8) = 1 if the segment
 *   eye[pair_f[i]] -> pos[pair_s[i]] is unoccluded under the occlusion mode in
 *   `flags` (Sec. 3.2.2), 0 if occluded, 2 if an index is out of range.
 *   tri / mesh as in accumulate_density.  gaze [n_eyes][3] (device, may be NULL):
 *   with it, each pair is tested with the arithmetic accumulate_density gives that
 *   pair (the segment's shear axis follows the fixation's gaze), so the answers are
 *   the density kernel's own; without it, the segment's own dominant axis.
 */
gm_status gm_debug_pair_values(const float* pos, int64_t n_points, const gm_fixations* fix,
                               double theta_deg, const int32_t* pair_s, const int32_t* pair_f,
                               int64_t m, float* g_out, void* stream);
gm_status gm_debug_sqrt_f64(const double* x, double* y, int64_t n, void* stream);
gm_status gm_debug_pair_visibility(gm_scene* scene, const float* pos, const int32_t* tri,
                                   const int32_t* mesh, int64_t n_points, const float* eye, const float* gaze,
                                   int32_t n_eyes, const int32_t* pair_s, const int32_t* pair_f,
                                   int64_t m, uint32_t flags, uint8_t* vis_out, void* stream);

/* ------------------------------------------------------------------------ */
/* Incremental maps and time windows.  rho is a sum over fixations, so a map */
/* over a fixed set of points can take its fixations in blocks (a recording  */
/* that grows, or several recordings) and any subset of them, such as those  */
/* whose start time falls in an analysis window (the time interval among    */
/* the generation parameters of Sec. 3.3.4; Sec. 2.3.3 asks for it).  A     */
/* gm_map holds the points in                                                */
/* their spatial order and one 64-bit fixed-point accumulator per point; the */
/* scale 2^S is fixed at creation from a budget D on the total duration of   */
/* the fixations it will take (S = 62 - e, 2^(e-1) <= 2 D / (sigma sqrt(2pi)) */
/* < 2^e), so every block is added exactly: a map fed blocks A then B holds  */
/* the same bits as one fed A u B in one call, in any order and split.        */
/* Values match accumulate_density's to the fixed-point quantum 2^-S (the two */
/* scales differ); visibility and cone decisions are the same code.           */
/* ------------------------------------------------------------------------ */
typedef struct gm_map gm_map;

/* Flag of gm_map_create: the meshes move; every fixation comes with each mesh's
 * pose at its time (gm_map_add_posed). */
#define GM_MAP_POSED 4u

/*
 * gm_map_create -- a map over n points with fixed theta and occlusion mode.
 * pos / tri / mesh: device, as in accumulate_density; read during the call (the
 * map keeps its own sorted copy).  theta_deg in (0, 45); flags: one GM_OCC_* mode,
 * optionally | GM_MAP_POSED.  A posed map holds points in their mesh's own frame
 * (the scene's coordinates are each mesh's own), needs mesh [n] with the points
 * grouped by mesh in mesh order (as the samplers write them; checked, blocking),
 * and with occlusion builds one BVH per mesh on the host on first use per scene
 * (blocking, kept by the scene).
 * max_total_duration: D in seconds, (0, 1e9]; fixations beyond it are refused
 * (see gm_map_add).  The map starts empty (all zero).  Allocates device memory
 * for about 40 bytes per point.  Queued on `stream`, then returns.  The scene
 * must outlive the map (its BVH answers the visibility of every block).
 */
gm_status gm_map_create(gm_scene* scene, const float* pos, const int32_t* tri, const int32_t* mesh,
                        int64_t n, double theta_deg, uint32_t flags, double max_total_duration,
                        gm_map** out, void* stream);

/*
 * gm_map_add -- accumulate a block of fixations.  time: device float64 [fix->n]
 * start time of each fixation (any clock), or NULL to take every fixation; with
 * time, fixation f is taken iff t_begin <= time[f] < t_end (NaN is never taken).
 * A taken fixation that is invalid (non-finite eye or gaze, zero gaze, duration
 * negative, non-finite or above 1e6 s) contributes nothing, as in
 * accumulate_density, and is counted as invalid.  Durations are charged to the
 * budget D rounded up to units of 2^-10 s; a fixation that does not fit in what
 * is left is not added and is counted as over budget (which ones, when a block
 * overruns the budget, is unspecified).  Queued on `stream`; the fixation arrays
 * must stay valid until the work completes.  The block's fixations
 * are selected and recorded on `stream` at once; their density work is gathered
 * with that of later blocks (up to 65,536 fixations, a larger block runs alone)
 * and runs in one launch at the next gm_map_read, on that call's stream.  Each add
 * records an event that the next add and the gathered launch wait for, so adds and
 * the read may come on different streams.  The sum is the same, bit for bit.
 */
gm_status gm_map_add(gm_map* map, const gm_fixations* fix, const double* time, double t_begin,
                     double t_end, void* stream);

/*
 * gm_map_add_posed -- accumulate a block of fixations on a posed map (dynamic
 * objects: the values stay bound to each object, Sec. 2.1 and Sec. 3.3.3).
 * pose: device float32 [fix->n][n_meshes][12], row-major 3x4 (A | b) taking mesh
 * m's own frame to the world at fixation f's time; A must be a similarity (a
 * rotation, possibly with a reflection, times a uniform scale): with s2 =
 * trace(A^T A) / 3 every entry of A^T A - s2 I must be within 1e-5 s2, else the
 * fixation is invalid.  Seen from mesh m, fixation f has eye A^-1 (e - b) and
 * gaze A^-1 r (A^-1 = A^T / s2), each evaluated in FP64 as ((A_0i v_0 +
 * A_1i v_1) + A_2i v_2) / s2 and rounded to FP32; the pair value of Sec. 3.2.1 is
 * computed in that frame (a similarity keeps angles, so g is the world's).
 * Visibility: GM_OCC_SELF tests the point's own mesh in its own frame;
 * GM_OCC_FULL also every other mesh, with the segment taken into that mesh's frame
 * (its parameter tau does not change).  time / window / budget / invalid
 * fixations as in gm_map_add.  Queued on `stream`.
 */
gm_status gm_map_add_posed(gm_map* map, const gm_fixations* fix, const float* pose, const double* time,
                           double t_begin, double t_end, void* stream);

/*
 * gm_map_read -- the map as accumulate_density's outputs (device, each may be
 * NULL): density [n] = rho in the caller's point order, density_norm [n] =
 * rho / max rho (all zero when the map is empty), max_out [1].  Queued.
 */
gm_status gm_map_read(gm_map* map, float* density, float* density_norm, float* max_out, void* stream);

/* gm_map_reset -- back to empty, with the whole budget.  Queued. */
gm_status gm_map_reset(gm_map* map, void* stream);

/*
 * gm_map_info -- host int64 out[4] = {fixations added, taken but invalid,
 * taken but over budget, budget used in units of 2^-10 s} since creation or the
 * last reset.  Blocking (synchronises the device).
 */
gm_status gm_map_info(gm_map* map, int64_t* out);
gm_status gm_map_destroy(gm_map* map);

/* ------------------------------------------------------------------------ */
/* The paper's own visibility approximation (Sec. 3.2.2, Sec. 3.3.2,        */
/* Appendix A), to measure it against the exact test of accumulate_density.  */
/* Per fixation: a camera at the eye looking along the head direction (the  */
/* gaze when none is given), with the world's up (0, 1, 0) ((0, 0, 1) for a */
/* vertical view); its view cropped to the bounds of the ellipse where the  */
/* 4-sigma cone meets the near plane (Appendix A: the gaze turned by -+phi, */
/* phi = atan(4 sigma), about u1 = r x i and u2 = r x u1 gives A0, A1, B0,  */
/* B1; E the gaze's hit; a = |A1 - A0| / 2, b = |B1 - B0| / 2, alpha the    */
/* angle of ME to the right vector; l', r' = E_x -+ sqrt(a^2 cos^2 alpha +  */
/* b^2 sin^2 alpha), b', t' = E_y -+ sqrt(a^2 sin^2 alpha + b^2 cos^2       */
/* alpha)); a resolution x resolution z-buffer holding, per pixel, the depth */
/* (distance along the forward axis) of the nearest surface of the whole    */
/* scene met by the ray through the pixel centre within [near, far] (+inf: */
/* none); CDNA4 has no raster hardware, so each pixel is one ray over the   */
/* scene BVH.  A sample inside the cropped frustum (the NDC cube) whose     */
/* depth D satisfies D - zbuf(its pixel) <= depth_eps D adds the angular   */
/* Gaussian of Sec. 3.2.1 (not cut at 4 sigma).  A fixation whose crop is  */
/* undefined (the cone reaches behind the camera) or whose crop corners lie */
/* 80 degrees or more off its gaze contributes nothing.  theta_deg must be */
/* in (0, 10].                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t resolution;  /* pixels per side, a multiple of 8 in [8, 1024] */
    float depth_eps;     /* relative depth tolerance, in [0, 1] */
    float near_plane;    /* metres, > 0 */
    float far_plane;     /* metres, > near_plane, finite */
    const float* head;   /* device [n][3] head view direction per fixation, or NULL (the gaze) */
} gm_zbuffer_params;

/* gm_render_zbuffers -- the z-buffers alone: zbuf device float [fix->n][R][R],
 * row j (along up) then column i (along right), pixel centre at NDC
 * (-1 + (2i + 1) / R, -1 + (2j + 1) / R).  Queued on `stream`. */
gm_status gm_render_zbuffers(gm_scene* scene, const gm_fixations* fix, double theta_deg,
                             const gm_zbuffer_params* params, float* zbuf, void* stream);

/* accumulate_density_zbuffer -- the density map with the approximation above in
 * place of the exact cone and segment test; outputs as accumulate_density.  The
 * scene holds the z-buffers meanwhile (4 R^2 bytes per fixation).  Queued. */
gm_status accumulate_density_zbuffer(gm_scene* scene, const float* pos, int64_t n, const gm_fixations* fix,
                                     double theta_deg, const gm_zbuffer_params* params, float* density,
                                     float* density_norm, float* max_out, void* stream);

/*
 * Export format (Sec. 3.3.3): one record per sample, ready for external analysis.
 * 48 bytes, little-endian, no padding.
 */
typedef struct {
    float value;       /* rho */
    float value_norm;  /* rho / max rho (NaN when not given) */
    int32_t mesh;      /* object (-1: unknown) */
    int32_t triangle;  /* triangle index within its mesh (-1: unknown) */
    float bary[2];     /* barycentric coordinates (b1, b2) of vertices 1 and 2; b0 = 1 - b1 - b2 */
    float local[3];    /* position in the mesh's own frame (the scene's coordinates) */
    float world[3];    /* position in the world: the mesh's pose applied to `local` */
} gm_export_record;

/*
 * gm_export_samples -- pack n samples into records.  Device inputs: tri [n]
 * scene-global triangle, mesh [n] or NULL (then from tri), bary [n][2], pos [n][3]
 * (as the samplers write them), density [n], density_norm [n] or NULL; pose:
 * device float32 [n_meshes][12] row-major 3x4 (A | b), the frame of each mesh in
 * the world at the time of interest, or NULL (world = local).  world = A local + b
 * in FP64, rounded.  out: device gm_export_record [n].  Queued on `stream`.
 */
gm_status gm_export_samples(gm_scene* scene, const int32_t* tri, const int32_t* mesh, const float* bary,
                            const float* pos, const float* density, const float* density_norm,
                            const float* pose, int64_t n, gm_export_record* out, void* stream);

/* ------------------------------------------------------------------------ */
/* Neural density field.  Not part of the paper's method: a Fourier-feature   */
/* MLP that learns the normalised map from (sample position, rho / max rho)  */
/* pairs produced by build_surface_samples + accumulate_density, and answers */
/* density queries at arbitrary surface points.  Network: 96 features        */
/* [sin, cos](2 pi f_b x~_a), f_b = max_cycles^(b/15), b = 0..15, x~ =        */
/* (x - lo) / ext in the                                                     */
/* scene's bounding cube -> 4 x (64, ReLU) -> 1 -> softplus; bf16 matrix-core */
/* products with fp32 accumulation; Adam on fp32 master weights.  Parameters */
/* (18,753 floats, host order): W1 [96][64] (input, output), b1 [64], W2, b2, */
/* W3, b3, W4, b4 (64 x 64, 64), w5 [64], b5; feature index 6 b + 2 a + c   */
/* (c = 0 sin, 1 cos).  The plain accumulation stays the fallback and the    */
/* reference for the field's error: a mesh whose held-out relative L2 error   */
/* exceeds max_rel_l2 (or a                                                  */
/* field never trained, or with a non-finite error) is answered by           */
/* accumulate_density at the query points.                                    */
/* ------------------------------------------------------------------------ */
typedef struct gm_field gm_field;

typedef struct {
    int32_t steps;       /* Adam steps */
    int32_t batch;       /* points per step, drawn with replacement from the training split */
    float lr;            /* initial learning rate, cosine-decayed to lr_final */
    float lr_final;
    float beta1, beta2, eps;
    float holdout;       /* fraction of points held out (per point, Philox hash of its index) */
    float max_rel_l2;    /* gate threshold on the per-mesh held-out relative L2 error */
    float target_max;    /* raw density that a target of 1 stands for (used by the fallback) */
    uint64_t seed;       /* key of the split and of the batch draws */
} gm_train_params;

#define GM_FIELD_PARAMS 18753

/* gm_field_create: one network per mesh, network m over mesh m's bounding cube
 * (corner at the box's lower corner, edge = its largest side), He-uniform weights
 * drawn from `seed` and m (zero biases); every mesh gate closed until trained.  The
 * band frequencies are f_b = max_cycles^(b / 15) cycles per cube edge, b = 0..15
 * (max_cycles <= 0: 32).  Blocking. */
gm_status gm_field_create(gm_scene* scene, uint64_t seed, double max_cycles, gm_field** out);
gm_status gm_field_destroy(gm_field* field);
/* host float [n_meshes][GM_FIELD_PARAMS] in, out (blocking) */
gm_status gm_field_set_params(gm_field* field, const float* params);
gm_status gm_field_get_params(gm_field* field, float* params);
/*
 * gm_field_train: pos [n][3], mesh [n] (mesh of each point, device) and target [n]
 * (device, the normalised density in [0, 1]).  For every mesh, runs `steps` Adam
 * steps of mean squared error of its network on its points of the training split,
 * then evaluates the mesh's relative L2 error sqrt(sum (y - t)^2 / sum t^2) on its
 * held-out points and opens the gate of the meshes at or below max_rel_l2.  The
 * gradients of a step are summed in a fixed order (no floating-point atomics), so
 * training gives the same weights, errors and gates on every run.  Blocking.
 */
gm_status gm_field_train(gm_field* field, const float* pos, const int32_t* mesh, const float* target,
                         int64_t n, const gm_train_params* params, void* stream);
/* host outputs (each may be NULL): rel_l2 [n_meshes] (NaN where a mesh had no held-out
 * point), gate [n_meshes] (1 = field answers), final training loss, steps done. */
gm_status gm_field_info(gm_field* field, float* rel_l2, uint8_t* gate, double* loss, int64_t* steps);
/* The field's value (softplus output) at q points, device pos [q][3] -> out [q], each
 * point by the network of its mesh (device mesh [q]; may be NULL for a one-mesh
 * scene), whatever the gates say; points of no mesh are left untouched; queued on
 * `stream`. */
gm_status gm_field_predict(gm_field* field, const float* pos, const int32_t* mesh, int64_t q, float* out,
                           void* stream);
/* One forward and backward pass of network `net` over all n points, n in (0, 65536] (no
 * update): the mean-squared-error gradient (host float [GM_FIELD_PARAMS]) and loss, summed
 * in a fixed order (the same bits on every call).  Blocking.  For gradient checks. */
gm_status gm_field_gradient(gm_field* field, int32_t net, const float* pos, const float* target, int64_t n,
                            float* grad, double* loss);

/*
 * gm_debug_adam_step -- one Adam update (Kingma and Ba 2015), the training loop's own
 * kernel, on count parameters (device float32, updated in place):
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   params -= lr (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps),
 * then grad is zeroed (as after each training step).  step counts from 1 and is
 * the update's number, which sets the bias corrections.  For checks of the
 * optimiser over several steps.  Queued on `stream`.
 */
gm_status gm_debug_adam_step(float* params, float* m, float* v, float* grad, int64_t count, int32_t step, float lr,
                             float beta1, float beta2, float eps, void* stream);

/*
 * query_density -- the normalised density at q query points (device pos [q][3];
 * tri / mesh [q] as in accumulate_density, at least one of them for the per-mesh
 * gate).  With a trained field, points of meshes whose gate is open get the
 * field's value; every other point (and every point when field is NULL) gets the
 * plain accumulation (fixations, theta_deg, flags as in accumulate_density)
 * divided by ref_max (> 0), else by the field's target_max, else by the largest
 * plain value among the query points.  out [q] (device float); used_fallback [q]
 * (device uint8, may be NULL) = 1 where the plain path answered.  Blocking when the
 * plain path runs (one count read-back).
 */
gm_status query_density(gm_field* field, gm_scene* scene, const gm_fixations* fix, double theta_deg,
                        uint32_t flags, const float* pos, const int32_t* tri, const int32_t* mesh, int64_t q,
                        double ref_max, float* out, uint8_t* used_fallback, void* stream);

/* ------------------------------------------------------------------------ */
/* Batched sessions: many maps (each a scene, its points and its fixations)   */
/* in one persistent launch.  Not in the paper; the per-map arithmetic is     */
/* exactly accumulate_density's (fixed-point sums, so each map is bit-equal   */
/* to its plain call).                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    gm_scene* scene;
    const float* pos;        /* device [n][3] */
    const int32_t* tri;      /* device [n] or NULL */
    const int32_t* mesh;     /* device [n] or NULL */
    int64_t n;
    gm_fixations fix;        /* device */
    double theta_deg;
    uint32_t flags;          /* GM_OCC_* */
    float* density;          /* device outputs [n], [n], [1]; each may be NULL */
    float* density_norm;
    float* max_out;
} gm_session;

typedef struct gm_batch gm_batch;

/*
 * gm_batch_create -- plan a batch and capture it in a HIP graph.  The work queue
 * holds one item per (session, tile of 256 * samples-per-lane sorted samples,
 * chunk of fixations), sorted by estimated cost, largest first; a persistent
 * kernel pulls items until the queue is empty.  The tile configuration (samples
 * per lane in {1, 2, 4}, LDS fixation block in {64, 128, 256}, fixations per
 * chunk) comes from the JSON cache `tune_cache` (NULL: the GM_TUNE_CACHE
 * environment variable; none: defaults) under a key built from the batch's
 * shape, or, with tune = 1, from timing candidates on this batch (coordinate
 * search), the winner being written back to the cache.  Every pointer of every
 * session must stay valid, with the same sizes, for the life of the batch; their
 * contents may change between runs.  Blocking (it runs the batch while planning).
 */
gm_status gm_batch_create(const gm_session* sessions, int32_t n_sessions, const char* tune_cache, int32_t tune,
                          gm_batch** out, void* stream);
/* Replay the captured graph on `stream`: every session's outputs are rewritten. */
gm_status gm_batch_run(gm_batch* batch, void* stream);
/* host outputs, each may be NULL: the chosen configuration (fixations per chunk 0 =
 * automatic per session), the number of work items, the tuned time of the queue kernel
 * in ms (-1 if not tuned), whether the configuration came from the cache */
gm_status gm_batch_info(const gm_batch* batch, int32_t* samples_per_lane, int32_t* fix_block,
                        int32_t* fix_per_chunk, int64_t* work_items, double* tuned_ms, int32_t* from_cache);
gm_status gm_batch_destroy(gm_batch* batch);

/*
 * gm_density_stats: counters of the last accumulate_density call on this scene,
 * host int64 out[4] = {pairs inside the 4-sigma cone, of those visible, packet
 * traversals of the BVH (one per wave, fixation and sample slot with at least one
 * in-cone lane), BVH node visits}.  Blocking (synchronises the device).
 */
gm_status gm_density_stats(gm_scene* scene, int64_t* out);

/* gm_density_counters: the same counters and more, host int64 out[n_out] = {the four
 * above, triangle tests (one per triangle tested by a packet for at least one of its
 * segments), in-cone pairs settled by the back-face rule (see gm_scene_mesh_closed),
 * fixations that the per-sample cone gate evaluated, summed over work items (a work item is
 * a tile of samples and a chunk of fixations; a fixation whose cone cannot reach the tile's
 * bounding sphere is skipped for the whole tile)}; entries past the known counters are set
 * to 0.  Blocking. */
gm_status gm_density_counters(gm_scene* scene, int64_t* out, int32_t n_out);

/*
 * Stage timing with HIP events recorded on the caller's stream around the
 * kernels of each stage (for measurement; off by default).
 * gm_profile_enable(scene, 1) starts recording and clears the totals.
 * gm_profile_read(scene, stage, total_ms, launches): blocking (waits for the
 * recorded events); stage is one of "sample" (a1-a3), "prep" (fixation records
 * and spatial sort), "density" (the gate / exact value / visibility kernel),
 * "finalize" (maximum and outputs).  Unknown stage: GM_ERR_INVALID_ARGUMENT.
 */
gm_status gm_profile_enable(gm_scene* scene, int32_t on);
gm_status gm_profile_read(gm_scene* scene, const char* stage, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* GAZEMAP_H */
