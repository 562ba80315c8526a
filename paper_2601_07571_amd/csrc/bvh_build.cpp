// bvh_build.cpp -- host construction of the occlusion BVH: binned surface-area
// heuristic (16 bins per axis over triangle centroids, Wald 2007), two child
// boxes per 64-byte node in depth-first order, 48-byte triangle records in leaf
// order.  Boxes are padded so that FP32 slab tests on the device never cull a
// box that a triangle hit lies in.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include "gm_internal.h"

namespace gm {

namespace {

constexpr int kBins = 16;
constexpr int kMaxDepth = 40;  // the traversal stack holds one entry per level, 64 at most

struct Box {
    float lo[3], hi[3];
    void reset()
    {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::numeric_limits<float>::infinity();
            hi[a] = -std::numeric_limits<float>::infinity();
        }
    }
    void grow(const float* p)
    {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], p[a]);
            hi[a] = std::max(hi[a], p[a]);
        }
    }
    void grow(const Box& b)
    {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], b.lo[a]);
            hi[a] = std::max(hi[a], b.hi[a]);
        }
    }
    double area() const
    {
        if (!(hi[0] >= lo[0])) return 0.0;
        const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

struct Builder {
    const float* V;
    const int32_t* I;
    const int32_t* tri_mesh;
    std::vector<Box> tbox;
    std::vector<float> cent;  // [T][3]
    std::vector<int32_t> idx;
    HostBvh* out;
    float pad_abs;
    int leaf_max = kLeafMax;

    Box range_box(int64_t b, int64_t e) const
    {
        Box bx;
        bx.reset();
        for (int64_t i = b; i < e; ++i) bx.grow(tbox[idx[i]]);
        return bx;
    }

    void padded(const Box& b, float* lo, float* hi) const
    {
        for (int a = 0; a < 3; ++a) {
            const float ext = b.hi[a] - b.lo[a];
            const float p = pad_abs + 1e-6f * ext;
            lo[a] = b.lo[a] - p;
            hi[a] = b.hi[a] + p;
        }
    }

    int32_t emit_leaf(int64_t b, int64_t e)
    {
        const int32_t first = (int32_t)out->tris.size();
        for (int64_t i = b; i < e; ++i) {
            const int32_t t = idx[i];
            BvhTri r;
            for (int k = 0; k < 3; ++k) {
                const float* p = V + 3 * (int64_t)I[3 * (int64_t)t + k];
                float* d = k == 0 ? r.v0 : (k == 1 ? r.v1 : r.v2);
                d[0] = p[0]; d[1] = p[1]; d[2] = p[2];
            }
            r.id = t;
            r.mesh = tri_mesh[t];
            r.pad = 0;
            out->tris.push_back(r);
        }
        return first;
    }

    // split [b, e) at the returned index (b < mid < e); `split_axis` receives the axis
    // along which the first part lies below the second (by centroid)
    int64_t split(int64_t b, int64_t e, int depth, int& split_axis)
    {
        const int64_t n = e - b;
        Box cb;
        cb.reset();
        for (int64_t i = b; i < e; ++i) cb.grow(&cent[3 * (int64_t)idx[i]]);
        int axis = 0;
        for (int a = 1; a < 3; ++a)
            if (cb.hi[a] - cb.lo[a] > cb.hi[axis] - cb.lo[axis]) axis = a;
        const bool degenerate = !(cb.hi[axis] > cb.lo[axis]);
        // guarantee depth <= kMaxDepth: object median when the range is too large for the depth left
        const bool force_median =
            degenerate || n > ((int64_t)leaf_max << std::min(40, std::max(0, kMaxDepth - 1 - depth)));
        if (!force_median) {
            double best = std::numeric_limits<double>::infinity();
            int best_axis = -1, best_bin = -1;
            for (int a = 0; a < 3; ++a) {
                const float ext = cb.hi[a] - cb.lo[a];
                if (!(ext > 0.0f)) continue;
                Box bb[kBins];
                int64_t cnt[kBins] = {0};
                for (int k = 0; k < kBins; ++k) bb[k].reset();
                const float scale = kBins / ext;
                for (int64_t i = b; i < e; ++i) {
                    const int32_t t = idx[i];
                    int k = (int)((cent[3 * (int64_t)t + a] - cb.lo[a]) * scale);
                    k = std::min(std::max(k, 0), kBins - 1);
                    cnt[k]++;
                    bb[k].grow(tbox[t]);
                }
                double left_area[kBins];
                int64_t left_cnt[kBins];
                Box acc;
                acc.reset();
                int64_t c = 0;
                for (int k = 0; k < kBins - 1; ++k) {
                    acc.grow(bb[k]);
                    c += cnt[k];
                    left_area[k] = acc.area();
                    left_cnt[k] = c;
                }
                acc.reset();
                c = 0;
                for (int k = kBins - 1; k >= 1; --k) {
                    acc.grow(bb[k]);
                    c += cnt[k];
                    const int64_t lc = left_cnt[k - 1];
                    if (lc == 0 || c == 0) continue;
                    const double cost = left_area[k - 1] * (double)lc + acc.area() * (double)c;
                    if (cost < best) {
                        best = cost;
                        best_axis = a;
                        best_bin = k;  // left = bins [0, k)
                    }
                }
            }
            if (best_axis >= 0) {
                const int a = best_axis;
                const float scale = kBins / (cb.hi[a] - cb.lo[a]);
                const float lo = cb.lo[a];
                auto it = std::partition(idx.begin() + b, idx.begin() + e, [&](int32_t t) {
                    int k = (int)((cent[3 * (int64_t)t + a] - lo) * scale);
                    k = std::min(std::max(k, 0), kBins - 1);
                    return k < best_bin;
                });
                const int64_t mid = it - idx.begin();
                if (mid > b && mid < e) {
                    split_axis = a;
                    return mid;
                }
            }
        }
        const int64_t mid = b + n / 2;
        split_axis = axis;
        if (!degenerate) {
            std::nth_element(idx.begin() + b, idx.begin() + mid, idx.begin() + e, [&](int32_t x, int32_t y) {
                return cent[3 * (int64_t)x + axis] < cent[3 * (int64_t)y + axis];
            });
        }
        return mid;
    }

    // builds an internal node over [b, e) (e - b > leaf_max) and returns its index
    int32_t build(int64_t b, int64_t e, int depth)
    {
        const int32_t id = (int32_t)out->nodes.size();
        out->nodes.emplace_back();
        out->depth = std::max(out->depth, depth + 1);
        int split_axis = 0;
        const int64_t mid = split(b, e, depth, split_axis);
        const int64_t rb[2] = {b, mid}, re[2] = {mid, e};
        BvhNode nd;
        std::memset(&nd, 0, sizeof(nd));
        for (int c = 0; c < 2; ++c) {
            const Box bx = range_box(rb[c], re[c]);
            float lo[3], hi[3];
            padded(bx, lo, hi);
            int32_t child, count;
            if (re[c] - rb[c] <= leaf_max) {
                child = ~emit_leaf(rb[c], re[c]);
                count = (int32_t)(re[c] - rb[c]);
                out->depth = std::max(out->depth, depth + 2);
            } else {
                child = build(rb[c], re[c], depth + 1);
                count = 0;
            }
            std::memcpy(c == 0 ? nd.lo0 : nd.lo1, lo, sizeof(lo));
            std::memcpy(c == 0 ? nd.hi0 : nd.hi1, hi, sizeof(hi));
            if (c == 0) { nd.child0 = child; nd.count0 = count; }
            else { nd.child1 = child; nd.count1 = count; }
        }
        nd.count0 |= split_axis << kSplitAxisShift;
        out->nodes[id] = nd;
        return id;
    }
};

}  // namespace

// V: all vertices [nv][3]; I: triangles with scene-global vertex indices [T][3].
void build_bvh(const float* V, const int32_t* I, const int32_t* tri_mesh, int64_t T, HostBvh& out, int leaf_max)
{
    Builder bd;
    bd.leaf_max = std::min(std::max(leaf_max, 1), kLeafMax);
    bd.V = V; bd.I = I; bd.tri_mesh = tri_mesh; bd.out = &out;
    bd.tbox.resize((size_t)T);
    bd.cent.resize((size_t)T * 3);
    bd.idx.resize((size_t)T);
    Box all;
    all.reset();
    for (int64_t t = 0; t < T; ++t) {
        Box& b = bd.tbox[(size_t)t];
        b.reset();
        for (int k = 0; k < 3; ++k) b.grow(V + 3 * (int64_t)I[3 * t + k]);
        for (int a = 0; a < 3; ++a) bd.cent[3 * t + a] = 0.5f * (b.lo[a] + b.hi[a]);
        bd.idx[(size_t)t] = (int32_t)t;
        all.grow(b);
    }
    float scale = 0.0f;
    for (int a = 0; a < 3; ++a) {
        out.lo[a] = all.lo[a];
        out.hi[a] = all.hi[a];
        scale = std::max(scale, std::max(std::fabs(all.lo[a]), std::fabs(all.hi[a])));
    }
    // FP32 slab arithmetic near coordinates of size `scale` is off by a few ulp
    bd.pad_abs = 4e-6f * scale + 1e-30f;
    out.nodes.clear();
    out.tris.clear();
    out.depth = 0;
    if (T > bd.leaf_max) {
        bd.build(0, T, 0);
    } else {
        // root with one leaf child and one empty child
        BvhNode nd;
        std::memset(&nd, 0, sizeof(nd));
        Box bx = bd.range_box(0, T);
        bd.padded(bx, nd.lo0, nd.hi0);
        nd.child0 = ~bd.emit_leaf(0, T);
        nd.count0 = (int32_t)T;
        for (int a = 0; a < 3; ++a) { nd.lo1[a] = 3.0e38f; nd.hi1[a] = -3.0e38f; }
        nd.child1 = -1;
        nd.count1 = 0;
        out.nodes.push_back(nd);
        out.depth = 2;
    }
    BvhTri pad;
    std::memset(&pad, 0, sizeof(pad));
    pad.id = -2;
    pad.mesh = -2;
    for (int k = 0; k < kLeafMax - 1; ++k) out.tris.push_back(pad);
}

void permute_tri_copies(const std::vector<BvhTri>& in, std::vector<BvhTri>& out)
{
    const size_t n = in.size();
    out.resize(kTriCopies * n);
    for (int c = 0; c < kTriCopies; ++c) {
        const int kz = c, kx = (c + 1) % 3, ky = (c + 2) % 3;
        for (size_t i = 0; i < n; ++i) {
            const BvhTri& t = in[i];
            BvhTri& r = out[c * n + i];
            r = t;
            r.v0[0] = t.v0[kx]; r.v0[1] = t.v0[ky]; r.v0[2] = t.v0[kz];
            r.v1[0] = t.v1[kx]; r.v1[1] = t.v1[ky]; r.v1[2] = t.v1[kz];
            r.v2[0] = t.v2[kx]; r.v2[1] = t.v2[ky]; r.v2[2] = t.v2[kz];
        }
    }
}

void octant_node_copies(const std::vector<BvhNode>& in, std::vector<BvhNode>& out)
{
    const size_t n = in.size();
    out.resize(kNodeCopies * n);
    for (int o = 0; o < kNodeCopies; ++o) {
        for (size_t i = 0; i < n; ++i) {
            BvhNode r = in[i];
            for (int a = 0; a < 3; ++a) {
                if (!((o >> a) & 1)) continue;
                std::swap(r.lo0[a], r.hi0[a]);
                std::swap(r.lo1[a], r.hi1[a]);
            }
            out[o * n + i] = r;
        }
    }
}

}  // namespace gm
