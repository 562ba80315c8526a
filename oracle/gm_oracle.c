/*
 * gm_oracle.c -- plain FP64 CPU oracle for surface-based fixation density maps
 * (Javerliat & Lavoue, "GPU accelerated surface-based gaze mapping for XR
 * experiences", arXiv 2601.07571).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP path.  Built with -O2 -ffp-contract=off and no fast-math so that
 * every FP64 operation below is a single IEEE round-to-nearest operation in
 * the order written.
 *
 * What it computes, step by step, in the paper's notation:
 *   - triangle area (Sec. 3.1.2, the area that feeds the adaptive sampling
 *     rule; written as half the cross-product norm, pinned against Heron);
 *   - area-proportional surface sampling (Sec. 3.1: samples per square metre
 *     independent of mesh resolution) as fixed-point area weights, an exact
 *     integer prefix sum, Philox4x32-10 counters and a square-root warp;
 *   - the paper's own per-triangle lattice sampler (Sec. 3.1.1 and 3.1.2,
 *     Eqs. 1-4: point count, index -> row/column, barycentrics, adaptive
 *     resolution);
 *   - the duration-weighted angular Gaussian of Sec. 3.2.1 (d1, d2, sigma,
 *     d, sigma_k, g), truncated at the 4-sigma cone (Sec. 3.2, Sec. 3.3.2);
 *   - visibility (Sec. 3.2.2) as an exact segment test eye -> sample against
 *     the occluding triangles (Moller-Trumbore in FP64), brute force or over
 *     the oracle's own median-split BVH;
 *   - normalisation by the maximum (Sec. 3.2.3).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the description in Salmon, Moraes, Dror and Shaw,    */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two */
/* 32x32->64 multiplications whose high halves are xored with the other two */
/* counter words and the round key; the key is bumped by the Weyl constants */
/* (golden ratio and sqrt(3)-1 in 32-bit fixed point) between rounds.       */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_MUL_A = 0xD2511F53u;
static const uint32_t PHILOX_MUL_B = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL_A = 0x9E3779B9u;
static const uint32_t PHILOX_WEYL_B = 0xBB67AE85u;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        uint64_t prod_a = (uint64_t)PHILOX_MUL_A * (uint64_t)x[0];
        uint64_t prod_b = (uint64_t)PHILOX_MUL_B * (uint64_t)x[2];
        uint32_t y0 = (uint32_t)(prod_b >> 32) ^ x[1] ^ k[0];
        uint32_t y1 = (uint32_t)prod_b;
        uint32_t y2 = (uint32_t)(prod_a >> 32) ^ x[3] ^ k[1];
        uint32_t y3 = (uint32_t)prod_a;
        x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
        k[0] += PHILOX_WEYL_A;
        k[1] += PHILOX_WEYL_B;
    }
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = x[3];
}

/* n consecutive counters (c0 + i, c1, c2, c3) as 64-bit increments of the low words. */
void or_philox_stream(uint64_t first, int64_t n, uint32_t w2, uint32_t w3,
                      uint64_t seed, uint32_t* out /* [n][4] */)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < n; ++i) {
        uint64_t j = first + (uint64_t)i;
        uint32_t ctr[4] = {(uint32_t)j, (uint32_t)(j >> 32), w2, w3};
        or_philox4x32_10(ctr, key, out + 4 * i);
    }
}

/* ------------------------------------------------------------------------ */
/* Triangle area (Sec. 3.1.2).  The paper evaluates it with Heron's formula; */
/* here it is half the norm of the edge cross product, the same quantity,   */
/* evaluated in one fixed FP64 order:                                       */
/*   u = v1 - v0, w = v2 - v0, c = u x w,                                   */
/*   A = 0.5 * sqrt((cx*cx + cy*cy) + cz*cz).                               */
/* ------------------------------------------------------------------------ */
static double tri_area_fp64(const float* a, const float* b, const float* c)
{
    double ux = (double)b[0] - (double)a[0];
    double uy = (double)b[1] - (double)a[1];
    double uz = (double)b[2] - (double)a[2];
    double wx = (double)c[0] - (double)a[0];
    double wy = (double)c[1] - (double)a[1];
    double wz = (double)c[2] - (double)a[2];
    double cx = uy * wz - uz * wy;
    double cy = uz * wx - ux * wz;
    double cz = ux * wy - uy * wx;
    double s = cx * cx + cy * cy;
    s = s + cz * cz;
    return 0.5 * sqrt(s);
}

void or_triangle_areas(const float* V, const int32_t* I, int64_t T, double* A)
{
    for (int64_t i = 0; i < T; ++i)
        A[i] = tri_area_fp64(V + 3 * (int64_t)I[3 * i], V + 3 * (int64_t)I[3 * i + 1],
                             V + 3 * (int64_t)I[3 * i + 2]);
}

/*
 * Fixed-point area weights of one mesh.  Sampling must put samples in
 * proportion to area (Sec. 3.1.2: a target number of samples per square
 * metre).  Areas are turned into integers W_i = floor(A_i * 2^S) with one
 * power-of-two scale per mesh, chosen from the largest area M and the
 * triangle count T so that the mesh total stays below 2^52:
 *   T*M = f * 2^e (f in [0.5, 1)),  S = 52 - e.
 * C is the inclusive prefix sum of W (exact integer arithmetic).
 * Returns the total W_m (= C[T-1]) and writes S.  A zero-area mesh gives 0.
 */
uint64_t or_mesh_weights(const double* A, int64_t T, uint64_t* W, uint64_t* C, int32_t* S_out)
{
    double M = 0.0;
    for (int64_t i = 0; i < T; ++i)
        if (A[i] > M) M = A[i];
    if (!(M > 0.0)) {
        for (int64_t i = 0; i < T; ++i) { W[i] = 0; C[i] = 0; }
        *S_out = 0;
        return 0;
    }
    int e = 0;
    (void)frexp((double)T * M, &e);
    int S = 52 - e;
    uint64_t run = 0;
    for (int64_t i = 0; i < T; ++i) {
        double scaled = floor(ldexp(A[i], S));
        W[i] = (uint64_t)scaled;
        run += W[i];
        C[i] = run;
    }
    *S_out = S;
    return run;
}

/* Samples of a mesh: round(k * area), with area = W_m * 2^-S. */
int64_t or_sample_count(uint64_t Wm, int32_t S, double k)
{
    double area = ldexp((double)Wm, -S);
    return (int64_t)floor(area * k + 0.5);
}

/*
 * Area-weighted sample placement for samples j in [j0, j0+n) of mesh `mesh_id`.
 * Counter (j_lo, j_hi, mesh_id, 0), key (seed_lo, seed_hi):
 *   U = x0 * 2^32 + x1, target = floor(U * W_m / 2^64),
 *   tri = smallest i with C_i > target          (triangle chosen with
 *                                                probability W_i / W_m);
 *   u = x2 / 2^32, v = x3 / 2^32, s = sqrt(u),
 *   (b0, b1, b2) = (1 - s, s (1 - v), s v)     (uniform in the triangle,
 *                                                Osada et al. 2002);
 *   P = (b0 v0 + b1 v1) + b2 v2 in FP64, rounded to FP32.
 * tri_out gets the mesh-local triangle index; bary_out (b1, b2) and pos_out
 * the FP64 values, pos32_out / bary32_out their FP32 roundings.
 */
void or_sample_mesh(const float* V, const int32_t* I, const uint64_t* C, int64_t T,
                    uint32_t mesh_id, uint64_t seed, int64_t j0, int64_t n,
                    int32_t* tri_out, double* bary_out, double* pos_out,
                    float* bary32_out, float* pos32_out)
{
    uint64_t Wm = C[T - 1];
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t s = 0; s < n; ++s) {
        uint64_t j = (uint64_t)(j0 + s);
        uint32_t ctr[4] = {(uint32_t)j, (uint32_t)(j >> 32), mesh_id, 0u};
        uint32_t x[4];
        or_philox4x32_10(ctr, key, x);
        uint64_t U = ((uint64_t)x[0] << 32) | (uint64_t)x[1];
        uint64_t target = (uint64_t)(((unsigned __int128)U * (unsigned __int128)Wm) >> 64);
        /* linear-time definition would be: first i with C[i] > target; bisection gives the same i */
        int64_t lo = 0, hi = T - 1;
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (C[mid] > target) hi = mid; else lo = mid + 1;
        }
        int64_t t = lo;
        double u = ldexp((double)x[2], -32);
        double v = ldexp((double)x[3], -32);
        double su = sqrt(u);
        double b1 = su * (1.0 - v);
        double b2 = su * v;
        double b0 = 1.0 - su;
        const float* p0 = V + 3 * (int64_t)I[3 * t];
        const float* p1 = V + 3 * (int64_t)I[3 * t + 1];
        const float* p2 = V + 3 * (int64_t)I[3 * t + 2];
        tri_out[s] = (int32_t)t;
        if (bary_out) { bary_out[2 * s] = b1; bary_out[2 * s + 1] = b2; }
        if (bary32_out) { bary32_out[2 * s] = (float)b1; bary32_out[2 * s + 1] = (float)b2; }
        for (int c = 0; c < 3; ++c) {
            double acc = b0 * (double)p0[c];
            acc = acc + b1 * (double)p1[c];
            acc = acc + b2 * (double)p2[c];
            if (pos_out) pos_out[3 * s + c] = acc;
            if (pos32_out) pos32_out[3 * s + c] = (float)acc;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* The paper's own sampler: a per-triangle lattice (Sec. 3.1.1, Sec. 3.1.2). */
/* A triangle subdivided at resolution r holds the points whose barycentric */
/* coordinates are multiples of 1/r; they are indexed row by row, row 0      */
/* holding one point and row `row` holding row + 1 points.                   */
/* ------------------------------------------------------------------------ */

/* Eq. (1): number of lattice points at resolution r, the triangular number */
/* (r + 1)(r + 2) / 2.                                                      */
int64_t or_lattice_points(int64_t r)
{
    return (r + 1) * (r + 2) / 2;
}

/*
 * Eq. (4): resolution giving k points per square metre on a triangle of area A.
 * Delta = 1 + 8 k A is the discriminant of r^2 + 3r + 2 - 2kA = 0; r = 1 when
 * Delta < 25, else the positive root (-3 + sqrt(Delta)) / 2.  Reading: the
 * paper's root is real while a subdivision needs a whole number; the root is
 * truncated, so a triangle never holds more than k A points (beyond the
 * three of the r = 1 floor).  Evaluated as Delta = (8 k) A + 1, in FP64.
 */
int64_t or_lattice_resolution(double k, double A)
{
    double delta = 8.0 * k;
    delta = delta * A;
    delta = delta + 1.0;
    if (!(delta >= 25.0)) return 1;
    double root = (sqrt(delta) - 3.0) / 2.0;
    return (int64_t)floor(root);
}

/*
 * Eq. (2): row and column of point idx.  row = ceil((-3 + sqrt(8 idx + 9)) / 2)
 * in FP64, then corrected with integers so that f(row - 1) <= idx < f(row)
 * holds exactly (f = Eq. (1)); col = idx - f(row - 1).
 */
void or_lattice_row_col(int64_t idx, int64_t* row, int64_t* col)
{
    int64_t r = (int64_t)ceil((sqrt(8.0 * (double)idx + 9.0) - 3.0) / 2.0);
    if (r < 0) r = 0;
    while (or_lattice_points(r) <= idx) ++r;
    while (r > 0 && or_lattice_points(r - 1) > idx) --r;
    *row = r;
    *col = idx - (r > 0 ? or_lattice_points(r - 1) : 0);
}

/* Per-triangle resolution and point count of a mesh; returns the total. */
int64_t or_lattice_counts(const float* V, const int32_t* I, int64_t T, double k, int64_t* r_out,
                          int64_t* count_out)
{
    int64_t total = 0;
    for (int64_t i = 0; i < T; ++i) {
        double A = tri_area_fp64(V + 3 * (int64_t)I[3 * i], V + 3 * (int64_t)I[3 * i + 1],
                                 V + 3 * (int64_t)I[3 * i + 2]);
        int64_t r = or_lattice_resolution(k, A);
        if (r_out) r_out[i] = r;
        if (count_out) count_out[i] = or_lattice_points(r);
        total += or_lattice_points(r);
    }
    return total;
}

/*
 * Every lattice point of a mesh, triangle by triangle, idx = 0 .. f(r) - 1 in
 * each.  Eq. (3) as printed, (col/r, 1 - row/r, 1 - (col + row)/r), does not
 * sum to one; the reading used keeps its first two weights and completes them:
 *   w1 = col / r, w2 = (r - row) / r, w3 = (row - col) / r
 * (each an exact integer ratio rounded once), which enumerates exactly the
 * lattice {(i, j, l) / r : i + j + l = r}.  P = (w1 v0 + w2 v1) + w3 v2 in FP64,
 * rounded to FP32.  bary32 holds (w2, w3), the weights of v1 and v2.
 * Writes at most `cap` points; returns the mesh total.
 */
int64_t or_lattice_mesh(const float* V, const int32_t* I, int64_t T, double k, int64_t cap,
                        int32_t* tri_out, double* pos_out, float* bary32_out, float* pos32_out)
{
    int64_t s = 0;
    for (int64_t i = 0; i < T; ++i) {
        const float* p0 = V + 3 * (int64_t)I[3 * i];
        const float* p1 = V + 3 * (int64_t)I[3 * i + 1];
        const float* p2 = V + 3 * (int64_t)I[3 * i + 2];
        double A = tri_area_fp64(p0, p1, p2);
        int64_t r = or_lattice_resolution(k, A);
        int64_t n = or_lattice_points(r);
        for (int64_t idx = 0; idx < n; ++idx, ++s) {
            if (s >= cap) continue;
            int64_t row, col;
            or_lattice_row_col(idx, &row, &col);
            double w1 = (double)col / (double)r;
            double w2 = (double)(r - row) / (double)r;
            double w3 = (double)(row - col) / (double)r;
            tri_out[s] = (int32_t)i;
            if (bary32_out) { bary32_out[2 * s] = (float)w2; bary32_out[2 * s + 1] = (float)w3; }
            for (int c = 0; c < 3; ++c) {
                double acc = w1 * (double)p0[c];
                acc = acc + w2 * (double)p1[c];
                acc = acc + w3 * (double)p2[c];
                if (pos_out) pos_out[3 * s + c] = acc;
                if (pos32_out) pos32_out[3 * s + c] = (float)acc;
            }
        }
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Visibility (Sec. 3.2.2).  A sample x is visible from eye e when no       */
/* occluding triangle other than the sample's own crosses the segment       */
/* e + tau (x - e) at 0 < tau < 1 - eps.  Triangle test: Moller-Trumbore in  */
/* FP64, inclusive edges, parallel (det == 0) is a miss.                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    double lo[3], hi[3];
    int32_t left, right;   /* children, or -1 */
    int32_t first, count;  /* leaf triangle range in `order` */
} or_node;

typedef struct or_scene {
    int64_t T;
    double* v;           /* [T][9] triangle vertices, FP64 (exact copies of FP32) */
    int32_t* tri_mesh;   /* [T] */
    int32_t* order;      /* [T] triangle ids in leaf order */
    or_node* nodes;
    int64_t n_nodes, cap_nodes;
} or_scene;

static void node_bounds(or_scene* sc, int32_t first, int32_t count, double lo[3], double hi[3])
{
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int32_t i = first; i < first + count; ++i) {
        const double* t = sc->v + 9 * (int64_t)sc->order[i];
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) {
                double c = t[3 * k + a];
                if (c < lo[a]) lo[a] = c;
                if (c > hi[a]) hi[a] = c;
            }
    }
    /* pad so that rounding in the box test can never cull a true hit */
    for (int a = 0; a < 3; ++a) {
        double pad = 1e-9 * (fabs(lo[a]) + fabs(hi[a]) + (hi[a] - lo[a])) + 1e-12;
        lo[a] -= pad; hi[a] += pad;
    }
}

static double centroid(const or_scene* sc, int32_t t, int a)
{
    const double* p = sc->v + 9 * (int64_t)t;
    return (p[a] + p[3 + a] + p[6 + a]) / 3.0;
}

static int32_t build_node(or_scene* sc, int32_t first, int32_t count)
{
    if (sc->n_nodes == sc->cap_nodes) {
        sc->cap_nodes = sc->cap_nodes ? 2 * sc->cap_nodes : 1024;
        sc->nodes = (or_node*)realloc(sc->nodes, sizeof(or_node) * (size_t)sc->cap_nodes);
    }
    int32_t id = (int32_t)sc->n_nodes++;
    or_node nd;
    node_bounds(sc, first, count, nd.lo, nd.hi);
    nd.left = nd.right = -1;
    nd.first = first; nd.count = count;
    if (count > 4) {
        /* median split of centroids along the widest centroid axis */
        double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int32_t i = first; i < first + count; ++i)
            for (int a = 0; a < 3; ++a) {
                double c = centroid(sc, sc->order[i], a);
                if (c < clo[a]) clo[a] = c;
                if (c > chi[a]) chi[a] = c;
            }
        int ax = 0;
        for (int a = 1; a < 3; ++a)
            if (chi[a] - clo[a] > chi[ax] - clo[ax]) ax = a;
        int32_t mid = count / 2;
        /* nth_element by quickselect on centroid[ax] */
        int32_t lo = first, hi = first + count - 1, k = first + mid;
        while (lo < hi) {
            double pivot = centroid(sc, sc->order[(lo + hi) / 2], ax);
            int32_t i = lo, j = hi;
            while (i <= j) {
                while (centroid(sc, sc->order[i], ax) < pivot) ++i;
                while (centroid(sc, sc->order[j], ax) > pivot) --j;
                if (i <= j) { int32_t tmp = sc->order[i]; sc->order[i] = sc->order[j]; sc->order[j] = tmp; ++i; --j; }
            }
            if (k <= j) hi = j; else if (k >= i) lo = i; else break;
        }
        nd.count = 0;
        sc->nodes[id] = nd;
        int32_t l = build_node(sc, first, mid);
        int32_t r = build_node(sc, first + mid, count - mid);
        sc->nodes[id].left = l;
        sc->nodes[id].right = r;
        return id;
    }
    sc->nodes[id] = nd;
    return id;
}

or_scene* or_scene_create(const float* V, const int32_t* I, const int32_t* tri_mesh, int64_t T)
{
    or_scene* sc = (or_scene*)calloc(1, sizeof(or_scene));
    sc->T = T;
    sc->v = (double*)malloc(sizeof(double) * 9 * (size_t)(T > 0 ? T : 1));
    sc->tri_mesh = (int32_t*)malloc(sizeof(int32_t) * (size_t)(T > 0 ? T : 1));
    sc->order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(T > 0 ? T : 1));
    for (int64_t t = 0; t < T; ++t) {
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a)
                sc->v[9 * t + 3 * k + a] = (double)V[3 * (int64_t)I[3 * t + k] + a];
        sc->tri_mesh[t] = tri_mesh[t];
        sc->order[t] = (int32_t)t;
    }
    if (T > 0) build_node(sc, 0, (int32_t)T);
    return sc;
}

void or_scene_destroy(or_scene* sc)
{
    if (!sc) return;
    free(sc->v); free(sc->tri_mesh); free(sc->order); free(sc->nodes);
    free(sc);
}

/* bookkeeping tolerances for "fragile" decisions (comparison only) */
static const double FRAG_BARY = 1e-4;
static const double FRAG_TAU = 1e-5;

/* Moller-Trumbore in FP64.  Returns 1 on a hit with 0 < tau < 1-eps (edges
 * inclusive), 0 otherwise; sets *near when the decision sits within the
 * bookkeeping tolerances of flipping. */
static int seg_tri(const double o[3], const double d[3], const double* t, double eps, int* near)
{
    double e1[3] = {t[3] - t[0], t[4] - t[1], t[5] - t[2]};
    double e2[3] = {t[6] - t[0], t[7] - t[1], t[8] - t[2]};
    double pv[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
    *near = 0;
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    double tv[3] = {o[0] - t[0], o[1] - t[1], o[2] - t[2]};
    double u = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
    double qv[3] = {tv[1] * e1[2] - tv[2] * e1[1], tv[2] * e1[0] - tv[0] * e1[2], tv[0] * e1[1] - tv[1] * e1[0]};
    double v = (d[0] * qv[0] + d[1] * qv[1] + d[2] * qv[2]) * inv;
    double tau = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
    double w = 1.0 - u - v;
    double tmax = 1.0 - eps;
    int hit = (u >= 0.0 && v >= 0.0 && w >= 0.0 && tau > 0.0 && tau < tmax);
    int inside_loose = (u >= -FRAG_BARY && v >= -FRAG_BARY && w >= -FRAG_BARY &&
                        tau > -FRAG_TAU && tau < tmax + FRAG_TAU);
    int inside_tight = (u >= FRAG_BARY && v >= FRAG_BARY && w >= FRAG_BARY &&
                        tau > FRAG_TAU && tau < tmax - FRAG_TAU);
    *near = inside_loose && !inside_tight;
    return hit;
}

static int seg_box(const double o[3], const double d[3], const double lo[3], const double hi[3], double tmax)
{
    double t0 = 0.0, t1 = tmax;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < lo[a] || o[a] > hi[a]) return 0;
            continue;
        }
        double ta = (lo[a] - o[a]) / d[a];
        double tb = (hi[a] - o[a]) / d[a];
        if (ta > tb) { double x = ta; ta = tb; tb = x; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
        if (t0 > t1) return 0;
    }
    return 1;
}

/* mode: 0 = no occlusion, 1 = own mesh occludes, 2 = every mesh occludes.
 * Returns 1 when visible.  *fragile (optional) = some triangle's decision is
 * within the bookkeeping tolerances and no triangle occludes robustly. */
int or_visible(const or_scene* sc, const double e[3], const double x[3], int32_t own_tri,
               int32_t own_mesh, int mode, double eps, int brute, int* fragile)
{
    if (fragile) *fragile = 0;
    if (mode == 0 || sc->T == 0) return 1;
    double d[3] = {x[0] - e[0], x[1] - e[1], x[2] - e[2]};
    int any_hit = 0, any_near = 0, robust_hit = 0;
    int32_t stack[256];
    int sp = 0;
    int64_t lin = 0;
    if (!brute) stack[sp++] = 0;
    for (;;) {
        int32_t first, count;
        if (brute) {
            if (lin >= sc->T) break;
            first = (int32_t)lin; count = (int32_t)((sc->T - lin) < 1024 ? (sc->T - lin) : 1024);
            lin += count;
        } else {
            if (sp == 0) break;
            const or_node* nd = &sc->nodes[stack[--sp]];
            if (!seg_box(e, d, nd->lo, nd->hi, 1.0 + FRAG_TAU)) continue;
            if (nd->left >= 0) {
                stack[sp++] = nd->left;
                stack[sp++] = nd->right;
                continue;
            }
            first = nd->first; count = nd->count;
        }
        for (int32_t i = first; i < first + count; ++i) {
            int32_t t = brute ? i : sc->order[i];
            if (t == own_tri) continue;
            if (mode == 1 && sc->tri_mesh[t] != own_mesh) continue;
            int near = 0;
            int h = seg_tri(e, d, sc->v + 9 * (int64_t)t, eps, &near);
            if (h && !fragile) return 0;      /* no bookkeeping asked: first hit decides */
            if (h) any_hit = 1;
            if (near) any_near = 1;
            if (h && !near) robust_hit = 1;
            if (robust_hit) { *fragile = 0; return 0; }
        }
    }
    if (fragile) *fragile = any_near;
    return any_hit ? 0 : 1;
}

/* ------------------------------------------------------------------------ */
/* The angular Gaussian of one (sample, fixation) pair, Sec. 3.2.1, in the   */
/* paper's notation.  p = x - e, d1 = p.r/|r| (scalar projection), d2 = the  */
/* scalar rejection |p x r|/|r|, sigma = tan(theta), d = d1 tan(theta),      */
/* sigma_k = (d2/d) sigma, g = t/(sigma sqrt(2 pi)) exp(-sigma_k^2/(2 sigma^2)).*/
/* Values propagate only inside the 4-sigma cone, sigma_k <= 4 sigma.        */
/* Pairs with d <= 0 (sample at or behind the eye plane) give nothing.       */
/* Returns 1 inside the cone and writes g; *margin (optional) gets          */
/* 1 - (sigma_k / 4 sigma)^2, the relative distance to the cone boundary.    */
/* ------------------------------------------------------------------------ */
int or_pair_value(const double x[3], const double e[3], const double r[3], double t,
                  double sigma, double* g_out, double* margin)
{
    double p[3] = {x[0] - e[0], x[1] - e[1], x[2] - e[2]};
    double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double rh[3] = {r[0] / rn, r[1] / rn, r[2] / rn};
    double d1 = p[0] * rh[0] + p[1] * rh[1] + p[2] * rh[2];
    double cx = p[1] * rh[2] - p[2] * rh[1];
    double cy = p[2] * rh[0] - p[0] * rh[2];
    double cz = p[0] * rh[1] - p[1] * rh[0];
    double d2 = sqrt(cx * cx + cy * cy + cz * cz);
    double d = d1 * sigma;
    *g_out = 0.0;
    if (margin) *margin = -INFINITY;
    if (!(d > 0.0)) return 0;
    double sigma_k = (d2 / d) * sigma;
    double ratio = sigma_k / (4.0 * sigma);
    if (margin) *margin = 1.0 - ratio * ratio;
    double g = t / (sigma * sqrt(2.0 * M_PI)) * exp(-(sigma_k * sigma_k) / (2.0 * sigma * sigma));
    *g_out = g;
    return sigma_k <= 4.0 * sigma;
}

/* ------------------------------------------------------------------------ */
/* Density of a set of samples (Sec. 3.2): rho_s = sum_f V(f,s) g(f,s) over  */
/* fixations inside the 4-sigma cone.  Threads split the samples statically. */
/* Per-sample bookkeeping (comparison only): budget = sum of g over pairs   */
/* whose gate margin is below 1e-5 or whose visibility is fragile; stats    */
/* [n][4] = in-cone pairs, visible pairs, ambiguous-gate pairs, fragile     */
/* visibility pairs.                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    const or_scene* sc;
    const float *pos, *eye, *gaze, *dur;
    const int32_t *tri, *mesh;
    int64_t n, F, begin, end;
    double sigma, eps;
    int mode, brute;
    double *rho, *budget;
    int64_t* stats;
} density_job;

static const double GATE_AMBIG = 1e-5;

static void* density_worker(void* arg)
{
    density_job* jb = (density_job*)arg;
    for (int64_t s = jb->begin; s < jb->end; ++s) {
        double x[3] = {jb->pos[3 * s], jb->pos[3 * s + 1], jb->pos[3 * s + 2]};
        double rho = 0.0, budget = 0.0;
        int64_t n_in = 0, n_vis = 0, n_amb = 0, n_frag = 0;
        for (int64_t f = 0; f < jb->F; ++f) {
            double e[3] = {jb->eye[3 * f], jb->eye[3 * f + 1], jb->eye[3 * f + 2]};
            double r[3] = {jb->gaze[3 * f], jb->gaze[3 * f + 1], jb->gaze[3 * f + 2]};
            double g, margin;
            int in = or_pair_value(x, e, r, (double)jb->dur[f], jb->sigma, &g, &margin);
            int ambiguous = fabs(margin) < GATE_AMBIG;
            if (!in && !ambiguous) continue;
            int fragile = 0;
            int vis = or_visible(jb->sc, e, x, jb->tri ? jb->tri[s] : -1, jb->mesh ? jb->mesh[s] : -1,
                                 jb->mode, jb->eps, jb->brute, &fragile);
            if (in) {
                ++n_in;
                if (vis) { ++n_vis; rho += g; }
            }
            if (ambiguous) ++n_amb;
            if (fragile && in) ++n_frag;
            if (ambiguous || (fragile && in)) budget += g;
        }
        jb->rho[s] = rho;
        if (jb->budget) jb->budget[s] = budget;
        if (jb->stats) {
            jb->stats[4 * s] = n_in; jb->stats[4 * s + 1] = n_vis;
            jb->stats[4 * s + 2] = n_amb; jb->stats[4 * s + 3] = n_frag;
        }
    }
    return NULL;
}

int or_density(const or_scene* sc, const float* pos, const int32_t* tri, const int32_t* mesh, int64_t n,
               const float* eye, const float* gaze, const float* dur, int64_t F, double theta_deg,
               int mode, double eps, int brute, int nthreads, double* rho, double* budget, int64_t* stats)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    double sigma = tan(theta_deg * M_PI / 180.0);
    density_job jobs[256];
    pthread_t th[256];
    int64_t chunk = (n + nthreads - 1) / nthreads;
    for (int i = 0; i < nthreads; ++i) {
        density_job* jb = &jobs[i];
        jb->sc = sc; jb->pos = pos; jb->eye = eye; jb->gaze = gaze; jb->dur = dur;
        jb->tri = tri; jb->mesh = mesh; jb->n = n; jb->F = F;
        jb->begin = i * chunk; jb->end = (i + 1) * chunk < n ? (i + 1) * chunk : n;
        jb->sigma = sigma; jb->eps = eps; jb->mode = mode; jb->brute = brute;
        jb->rho = rho; jb->budget = budget; jb->stats = stats;
        if (jb->begin >= jb->end) continue;
        if (nthreads == 1) { density_worker(jb); continue; }
        pthread_create(&th[i], NULL, density_worker, jb);
    }
    if (nthreads > 1)
        for (int i = 0; i < nthreads; ++i)
            if (jobs[i].begin < jobs[i].end) pthread_join(th[i], NULL);
    return 0;
}

/* Visibility of explicit (sample, fixation) pairs; vis/fragile are [m] bytes. */
void or_pair_visibility(const or_scene* sc, const float* pos, const int32_t* tri, const int32_t* mesh,
                        const float* eye, const int64_t* pair_s, const int64_t* pair_f, int64_t m,
                        int mode, double eps, int brute, uint8_t* vis, uint8_t* fragile)
{
    for (int64_t i = 0; i < m; ++i) {
        int64_t s = pair_s[i], f = pair_f[i];
        double x[3] = {pos[3 * s], pos[3 * s + 1], pos[3 * s + 2]};
        double e[3] = {eye[3 * f], eye[3 * f + 1], eye[3 * f + 2]};
        int fr = 0;
        vis[i] = (uint8_t)or_visible(sc, e, x, tri ? tri[s] : -1, mesh ? mesh[s] : -1, mode, eps, brute, &fr);
        if (fragile) fragile[i] = (uint8_t)fr;
    }
}

/* Normalisation (Sec. 3.2.3): divide by the maximum; all zero stays zero. */
double or_normalize(const double* rho, int64_t n, double* out)
{
    double mx = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (rho[i] > mx) mx = rho[i];
    for (int64_t i = 0; i < n; ++i) out[i] = mx > 0.0 ? rho[i] / mx : 0.0;
    return mx;
}

/* g and the gate margin for explicit (sample, fixation) pairs (no visibility). */
void or_pair_values(const float* pos, const float* eye, const float* gaze, const float* dur,
                    const int64_t* pair_s, const int64_t* pair_f, int64_t m, double theta_deg,
                    double* g_out, double* margin_out, uint8_t* in_out)
{
    double sigma = tan(theta_deg * M_PI / 180.0);
    for (int64_t i = 0; i < m; ++i) {
        int64_t s = pair_s[i], f = pair_f[i];
        double x[3] = {pos[3 * s], pos[3 * s + 1], pos[3 * s + 2]};
        double e[3] = {eye[3 * f], eye[3 * f + 1], eye[3 * f + 2]};
        double r[3] = {gaze[3 * f], gaze[3 * f + 1], gaze[3 * f + 2]};
        double g, mg;
        int in = or_pair_value(x, e, r, (double)dur[f], sigma, &g, &mg);
        g_out[i] = in ? g : 0.0;
        if (margin_out) margin_out[i] = mg;
        if (in_out) in_out[i] = (uint8_t)in;
    }
}

/* ------------------------------------------------------------------------ */
/* The paper's own visibility approximation (Sec. 3.2.2, Sec. 3.3.2,        */
/* Appendix A): per fixation, a z-buffer of the scene seen through a camera */
/* cropped to the 4-sigma cone; a sample inside the cropped frustum is      */
/* visible when its depth is within eps of the depth stored at its pixel.   */
/* The buffer holds, per pixel, the depth of the nearest surface met by the */
/* ray through the pixel centre (what rasterisation stores there).  Camera */
/* cam[13] = right (3), up (3), forward (3) unit vectors, then l', r', b',  */
/* t' of the crop on the near plane (Appendix A).  Depth = distance along   */
/* forward; the frustum keeps depths in [near, far].                        */
/* ------------------------------------------------------------------------ */

/* Nearest hit of o + t d with tmin <= t <= tmax over all triangles (MT in  */
/* FP64, inclusive edges); INFINITY when none.  *ambiguous = a triangle     */
/* within the bookkeeping band of a hit (its edges, or tmin / tmax) lies in */
/* front of or at the nearest hit, so a rasteriser could store its depth.   */
double or_closest(const or_scene* sc, const double o[3], const double d[3], double tmin, double tmax,
                  int* ambiguous)
{
    double best = INFINITY, best_band = INFINITY;
    int32_t stack[256];
    int sp = 0;
    if (sc->T > 0) stack[sp++] = 0;
    while (sp > 0) {
        const or_node* nd = &sc->nodes[stack[--sp]];
        /* box test on [0, min(tmax, best) (1 + band)] with the ray's own parameter */
        if (!seg_box(o, d, nd->lo, nd->hi, fmin(tmax, best) * (1.0 + FRAG_TAU))) continue;
        if (nd->left >= 0) {
            stack[sp++] = nd->left;
            stack[sp++] = nd->right;
            continue;
        }
        for (int32_t i = nd->first; i < nd->first + nd->count; ++i) {
            const double* t = sc->v + 9 * (int64_t)sc->order[i];
            double e1[3] = {t[3] - t[0], t[4] - t[1], t[5] - t[2]};
            double e2[3] = {t[6] - t[0], t[7] - t[1], t[8] - t[2]};
            double pv[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
            double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
            if (det == 0.0) continue;
            double inv = 1.0 / det;
            double tv[3] = {o[0] - t[0], o[1] - t[1], o[2] - t[2]};
            double u = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
            double qv[3] = {tv[1] * e1[2] - tv[2] * e1[1], tv[2] * e1[0] - tv[0] * e1[2], tv[0] * e1[1] - tv[1] * e1[0]};
            double v = (d[0] * qv[0] + d[1] * qv[1] + d[2] * qv[2]) * inv;
            double tt = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
            double w = 1.0 - u - v;
            if (u >= 0.0 && v >= 0.0 && w >= 0.0 && tt >= tmin && tt <= tmax && tt < best) best = tt;
            int loose = u >= -FRAG_BARY && v >= -FRAG_BARY && w >= -FRAG_BARY && tt >= tmin * (1.0 - FRAG_TAU) &&
                        tt <= tmax * (1.0 + FRAG_TAU);
            int tight = u >= FRAG_BARY && v >= FRAG_BARY && w >= FRAG_BARY && tt >= tmin * (1.0 + FRAG_TAU) &&
                        tt <= tmax * (1.0 - FRAG_TAU);
            if (loose && !tight && tt < best_band) best_band = tt;
        }
    }
    if (ambiguous) *ambiguous = best_band <= best * (1.0 + FRAG_TAU);
    return best;
}

/* z-buffer of one fixation: zbuf[j * R + i] for pixel column i (along the */
/* right vector) and row j (along up), centre at NDC (-1 + (2i + 1) / R,   */
/* -1 + (2j + 1) / R).  The ray through it has direction x' right + y' up + */
/* forward (depth = its parameter) with x' = (ndc_x + ox) / sx, sx = 2n /  */
/* (r' - l'), ox = (r' + l') / (r' - l'), the inverse of the crop matrix.  */
void or_zbuffer(const or_scene* sc, const double e[3], const double cam[13], double near_, double far_, int R,
                double* zbuf, uint8_t* amb)
{
    double sx = 2.0 * near_ / (cam[10] - cam[9]), ox = (cam[10] + cam[9]) / (cam[10] - cam[9]);
    double sy = 2.0 * near_ / (cam[12] - cam[11]), oy = (cam[12] + cam[11]) / (cam[12] - cam[11]);
    for (int j = 0; j < R; ++j)
        for (int i = 0; i < R; ++i) {
            double nx = -1.0 + (2.0 * i + 1.0) / R, ny = -1.0 + (2.0 * j + 1.0) / R;
            double xc = (nx + ox) / sx, yc = (ny + oy) / sy;
            double d[3];
            for (int a = 0; a < 3; ++a) d[a] = xc * cam[a] + yc * cam[3 + a] + cam[6 + a];
            int am = 0;
            zbuf[(int64_t)j * R + i] = or_closest(sc, e, d, near_, far_, &am);
            if (amb) amb[(int64_t)j * R + i] = (uint8_t)am;
        }
}

typedef struct {
    const or_scene* sc;
    const float *pos, *eye, *gaze, *dur;
    const double* cams;
    int64_t n, F, begin, end;
    double sigma, eps_depth, near_, far_;
    int R;
    const double* zbuf;    /* [F][R][R] */
    const uint8_t* zamb;
    double *rho, *budget;
    int64_t* stats;
} zdensity_job;

static const double ZB_NDC_BAND = 1e-5, ZB_PIX_BAND = 1e-4, ZB_DEPTH_BAND = 1e-5;

static void* zdensity_worker(void* arg)
{
    zdensity_job* jb = (zdensity_job*)arg;
    const int R = jb->R;
    for (int64_t s = jb->begin; s < jb->end; ++s) {
        double x[3] = {jb->pos[3 * s], jb->pos[3 * s + 1], jb->pos[3 * s + 2]};
        double rho = 0.0, budget = 0.0;
        int64_t n_in = 0, n_vis = 0, n_amb = 0;
        for (int64_t f = 0; f < jb->F; ++f) {
            const double* cam = jb->cams + 13 * f;
            double e[3] = {jb->eye[3 * f], jb->eye[3 * f + 1], jb->eye[3 * f + 2]};
            double r[3] = {jb->gaze[3 * f], jb->gaze[3 * f + 1], jb->gaze[3 * f + 2]};
            double p[3] = {x[0] - e[0], x[1] - e[1], x[2] - e[2]};
            double xc = p[0] * cam[0] + p[1] * cam[1] + p[2] * cam[2];
            double yc = p[0] * cam[3] + p[1] * cam[4] + p[2] * cam[5];
            double D = p[0] * cam[6] + p[1] * cam[7] + p[2] * cam[8];
            if (!(D > 0.0)) continue;
            double sx = 2.0 * jb->near_ / (cam[10] - cam[9]), ox = (cam[10] + cam[9]) / (cam[10] - cam[9]);
            double sy = 2.0 * jb->near_ / (cam[12] - cam[11]), oy = (cam[12] + cam[11]) / (cam[12] - cam[11]);
            double nx = sx * xc / D - ox, ny = sy * yc / D - oy;
            int in = D >= jb->near_ && D <= jb->far_ && fabs(nx) <= 1.0 && fabs(ny) <= 1.0;
            int amb_in = fabs(fabs(nx) - 1.0) <= ZB_NDC_BAND || fabs(fabs(ny) - 1.0) <= ZB_NDC_BAND ||
                         fabs(D - jb->near_) <= ZB_NDC_BAND * D || fabs(D - jb->far_) <= ZB_NDC_BAND * D;
            if (!in && !amb_in) continue;
            double g, margin;
            (void)or_pair_value(x, e, r, (double)jb->dur[f], jb->sigma, &g, &margin);
            if (!in) {
                budget += g;
                ++n_amb;
                continue;
            }
            double fx = (nx + 1.0) * 0.5 * R, fy = (ny + 1.0) * 0.5 * R;
            int i = (int)floor(fx), j = (int)floor(fy);
            if (i < 0) i = 0;
            if (i > R - 1) i = R - 1;
            if (j < 0) j = 0;
            if (j > R - 1) j = R - 1;
            double frx = fx - floor(fx), fry = fy - floor(fy);
            int amb_pix = (frx <= ZB_PIX_BAND || frx >= 1.0 - ZB_PIX_BAND || fry <= ZB_PIX_BAND ||
                           fry >= 1.0 - ZB_PIX_BAND) && fx > ZB_PIX_BAND && fx < R - ZB_PIX_BAND &&
                          fy > ZB_PIX_BAND && fy < R - ZB_PIX_BAND;
            int64_t px = ((int64_t)f * R + j) * R + i;
            double zb = jb->zbuf[px];
            double m = jb->eps_depth * D - (D - zb);
            int vis = isinf(zb) || m >= 0.0;
            int amb_d = (!isinf(zb) && fabs(m) <= ZB_DEPTH_BAND * D) || jb->zamb[px];
            ++n_in;
            if (vis) { ++n_vis; rho += g; }
            if (amb_in || amb_pix || amb_d) { budget += g; ++n_amb; }
        }
        jb->rho[s] = rho;
        jb->budget[s] = budget;
        if (jb->stats) {
            jb->stats[4 * s] = n_in; jb->stats[4 * s + 1] = n_vis;
            jb->stats[4 * s + 2] = n_amb; jb->stats[4 * s + 3] = 0;
        }
    }
    return NULL;
}

typedef struct {
    const or_scene* sc;
    const float* eye;
    const double* cams;
    double near_, far_;
    int R;
    int64_t f0, f1;
    double* zbuf;
    uint8_t* zamb;
} zbuf_job;

static void* zbuf_worker(void* arg)
{
    zbuf_job* jb = (zbuf_job*)arg;
    const int64_t RR = (int64_t)jb->R * jb->R;
    for (int64_t f = jb->f0; f < jb->f1; ++f) {
        double e[3] = {jb->eye[3 * f], jb->eye[3 * f + 1], jb->eye[3 * f + 2]};
        or_zbuffer(jb->sc, e, jb->cams + 13 * f, jb->near_, jb->far_, jb->R, jb->zbuf + f * RR, jb->zamb + f * RR);
    }
    return NULL;
}

/* Density with the z-buffer test: rho_s = sum over fixations whose cropped */
/* frustum holds s and whose z-buffer sees s of the Gaussian g (not cut at   */
/* 4 sigma: the frustum does the cutting).  zbuf / zamb: caller-owned       */
/* [F][R][R] (filled here).  budget = sum of g over pairs whose frustum,    */
/* pixel or depth decision sits within the bookkeeping bands.               */
int or_density_zbuffer(const or_scene* sc, const float* pos, int64_t n, const float* eye, const float* gaze,
                       const float* dur, const double* cams, int64_t F, double theta_deg, int R, double eps_depth,
                       double near_, double far_, int nthreads, double* zbuf, uint8_t* zamb, double* rho,
                       double* budget, int64_t* stats)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    zbuf_job zj[256];
    int64_t fc = (F + nthreads - 1) / nthreads;
    for (int i = 0; i < nthreads; ++i) {
        zj[i] = (zbuf_job){sc, eye, cams, near_, far_, R, i * fc, (i + 1) * fc < F ? (i + 1) * fc : F, zbuf, zamb};
        if (zj[i].f0 < zj[i].f1) pthread_create(&th[i], NULL, zbuf_worker, &zj[i]);
    }
    for (int i = 0; i < nthreads; ++i)
        if (zj[i].f0 < zj[i].f1) pthread_join(th[i], NULL);
    double sigma = tan(theta_deg * M_PI / 180.0);
    zdensity_job jobs[256];
    int64_t chunk = (n + nthreads - 1) / nthreads;
    for (int i = 0; i < nthreads; ++i) {
        zdensity_job* jb = &jobs[i];
        jb->sc = sc; jb->pos = pos; jb->eye = eye; jb->gaze = gaze; jb->dur = dur; jb->cams = cams;
        jb->n = n; jb->F = F; jb->begin = i * chunk; jb->end = (i + 1) * chunk < n ? (i + 1) * chunk : n;
        jb->sigma = sigma; jb->eps_depth = eps_depth; jb->near_ = near_; jb->far_ = far_; jb->R = R;
        jb->zbuf = zbuf; jb->zamb = zamb; jb->rho = rho; jb->budget = budget; jb->stats = stats;
        if (jb->begin < jb->end) pthread_create(&th[i], NULL, zdensity_worker, jb);
    }
    for (int i = 0; i < nthreads; ++i)
        if (jobs[i].begin < jobs[i].end) pthread_join(th[i], NULL);
    return 0;
}
