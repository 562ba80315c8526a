// mesh_topology.cpp -- host-side check that a triangle mesh bounds a solid, for the
// back-face rule of the visibility test.
//
// A mesh is taken as closed when, after merging vertices at identical positions, every
// directed edge (a, b) of its triangles occurs exactly once and its reverse (b, a)
// occurs exactly once (an edge-manifold surface without border, every triangle wound
// consistently with its neighbours), no triangle repeats a merged vertex, and its signed
// volume sum_t v0 . (v1 x v2) / 6 is positive (normals (v1 - v0) x (v2 - v0) point out).
// The winding number of such a surface about a point outside its bounding box is 0 and
// crossing a triangle against its normal raises it by one; self-intersection is not
// checked (a caller with such a mesh clears its flag, see gm_scene_set_mesh_closed).
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <utility>
#include <vector>

#include "gm_internal.h"

namespace gm {

bool mesh_is_closed(const float* V, int64_t nv, const int32_t* I, int64_t T)
{
    if (T < 4 || nv < 4) return false;
    // merge vertices at bit-identical positions
    struct Key {
        uint32_t x, y, z;
        bool operator<(const Key& o) const { return x != o.x ? x < o.x : (y != o.y ? y < o.y : z < o.z); }
        bool operator==(const Key& o) const { return x == o.x && y == o.y && z == o.z; }
    };
    std::vector<std::pair<Key, int64_t>> keys((size_t)nv);
    for (int64_t v = 0; v < nv; ++v) {
        Key k;
        float p[3] = {V[3 * v], V[3 * v + 1], V[3 * v + 2]};
        for (float& c : p)
            if (c == 0.0f) c = 0.0f;  // -0 and +0 are one position
        std::memcpy(&k.x, &p[0], 4);
        std::memcpy(&k.y, &p[1], 4);
        std::memcpy(&k.z, &p[2], 4);
        keys[(size_t)v] = {k, v};
    }
    std::sort(keys.begin(), keys.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    std::vector<int64_t> id((size_t)nv);
    int64_t next = -1;
    for (size_t i = 0; i < keys.size(); ++i) {
        if (i == 0 || !(keys[i].first == keys[i - 1].first)) ++next;
        id[(size_t)keys[i].second] = next;
    }
    // directed edges
    std::vector<uint64_t> e;
    e.reserve((size_t)(3 * T));
    double vol = 0.0;
    for (int64_t t = 0; t < T; ++t) {
        const int64_t a = id[(size_t)I[3 * t]], b = id[(size_t)I[3 * t + 1]], c = id[(size_t)I[3 * t + 2]];
        if (a == b || b == c || c == a) return false;
        e.push_back(((uint64_t)a << 32) | (uint64_t)b);
        e.push_back(((uint64_t)b << 32) | (uint64_t)c);
        e.push_back(((uint64_t)c << 32) | (uint64_t)a);
        const float* p0 = V + 3 * (int64_t)I[3 * t];
        const float* p1 = V + 3 * (int64_t)I[3 * t + 1];
        const float* p2 = V + 3 * (int64_t)I[3 * t + 2];
        const double cx = (double)p1[1] * p2[2] - (double)p1[2] * p2[1];
        const double cy = (double)p1[2] * p2[0] - (double)p1[0] * p2[2];
        const double cz = (double)p1[0] * p2[1] - (double)p1[1] * p2[0];
        vol += (double)p0[0] * cx + (double)p0[1] * cy + (double)p0[2] * cz;
    }
    if (next >= ((int64_t)1 << 32)) return false;
    std::sort(e.begin(), e.end());
    for (size_t i = 1; i < e.size(); ++i)
        if (e[i] == e[i - 1]) return false;  // a directed edge twice: not consistently wound
    for (uint64_t k : e) {
        const uint64_t rev = (k << 32) | (k >> 32);
        if (!std::binary_search(e.begin(), e.end(), rev)) return false;  // a border edge
    }
    return vol > 0.0;
}

}  // namespace gm

extern "C" int32_t gm_mesh_closed(const float* vertices, int32_t n_vertices, const int32_t* indices,
                                  int32_t n_triangles)
{
    if (!vertices || !indices || n_vertices < 0 || n_triangles < 0) return -1;
    for (int64_t t = 0; t < 3 * (int64_t)n_triangles; ++t)
        if (indices[t] < 0 || indices[t] >= n_vertices) return -1;
    return gm::mesh_is_closed(vertices, n_vertices, indices, n_triangles) ? 1 : 0;
}
