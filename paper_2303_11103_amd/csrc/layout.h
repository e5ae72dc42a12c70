// Device data layout shared by the host scene builder and the HIP kernels.
// Plain C++ (no HIP types) so that the host builder compiles with any C++17
// compiler.
#pragma once
#include <cstdint>

namespace rt {

// Binary BVH node holding the bounds of both children (one 64-byte line).
//   a = (lo0.x, hi0.x, lo0.y, hi0.y)   b = (lo1.x, hi1.x, lo1.y, hi1.y)
//   c = (lo0.z, hi0.z, lo1.z, hi1.z)   child[0], child[1]
// child >= 0: index of an inner node; child < 0: leaf ~((first << 5) | (count - 1))
// over the reordered triangle array, count <= 32.
struct alignas(64) Node {
    float a[4];
    float b[4];
    float c[4];
    int32_t child[2];
    int32_t pad[2];
};
static_assert(sizeof(Node) == 64, "node must be one cache line");

constexpr int kLeafShift = 5;
constexpr int kMaxLeaf = 1 << kLeafShift;  // 32
constexpr int kMaxDepth = 30;              // traversal stack is kMaxDepth + 2 deep

inline int32_t make_leaf(int32_t first, int32_t count) { return ~((first << kLeafShift) | (count - 1)); }

// Intersection record of one triangle in BVH leaf order (96 bytes, fp64).
// v0, e1 = v1 - v0, e2 = v2 - v0 computed exactly from the float32 input;
// thr = 1e-12 |e1| |e2| (parallel-ray threshold on |det| for unit directions).
struct alignas(32) Tri {
    double v0[3];
    double e1[3];
    double e2[3];
    double thr;
    int32_t face;   // face id (coplanar same-material group)
    int32_t orig;   // index in the caller's triangle array
    int32_t pad[2];
};
static_assert(sizeof(Tri) == 96, "triangle record size");

// Shading record per triangle in BVH leaf order: canonical unit normal (fp64)
// and material.
struct alignas(32) Shade {
    double n[3];
    int32_t mat;
    int32_t face;
};
static_assert(sizeof(Shade) == 32, "shade record size");

// Per-face data used by the image method.
struct alignas(32) Face {
    double n[3];      // canonical unit normal
    double q[3];      // a point of the plane (first vertex of its first triangle)
    int32_t mat;
    int32_t first;    // first entry in face_tris
    int32_t count;    // number of triangles
    int32_t pad;
};
static_assert(sizeof(Face) == 64, "face record size");

// Material constants derived on the host at the carrier frequency.
struct Mat {
    float eta_re, eta_im;      // complex relative permittivity eps_r - j sigma/(eps0 w)
    int32_t pec;               // perfect conductor
    int32_t pad;
    double eta_re_d, eta_im_d; // the same in fp64
};

}  // namespace rt
