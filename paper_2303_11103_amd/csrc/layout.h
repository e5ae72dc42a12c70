// Device data layout shared by the host scene builder and the HIP kernels.
// Plain C++ (no HIP types) so that the host builder compiles with any C++17
// compiler.
#pragma once
#include <cstdint>

namespace rt {

// 4-wide BVH node holding the bounds of its (up to) four children, child
// coordinates interleaved so that one 16-byte load fetches one bound of all
// four children (two 64-byte lines):
//   bx[0] = lo.x, bx[1] = hi.x, bx[2] = lo.y, bx[3] = hi.y, bz[0] = lo.z, bz[1] = hi.z
// child >= 0: index of an inner node; kEmptyChild: unused slot (its box has
// lo = +inf and hi = -inf on every axis, so every ray misses it); other
// negative values: leaf ~((first << 5) | (count - 1)) over the reordered
// triangle array, count <= 32.
struct alignas(128) Node {
    float bx[4][4];
    float bz[2][4];
    int32_t child[4];
    int32_t pad[4];
};
static_assert(sizeof(Node) == 128, "node must be two cache lines");

constexpr int32_t kEmptyChild = (int32_t)0x80000000;
constexpr int kLeafShift = 5;
constexpr int kMaxLeaf = 1 << kLeafShift;  // 32
constexpr int kMaxDepth = 30;              // binary build tree depth bound
#ifndef RT_LDS_STACK
#define RT_LDS_STACK 32
#endif
constexpr int kStackEntries = RT_LDS_STACK;         // traversal stack entries per lane kept in LDS
constexpr int kStackOverflow = 64 - RT_LDS_STACK;   // further entries per lane in private memory

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

// Wedge of the mesh for first-order diffraction: an edge shared by two
// triangles of different faces whose solid interior angle alpha is below pi.
// a: first vertex, e: unit edge direction, t0: unit vector in the 0-face
// (the face with the smaller id) orthogonal to e pointing into the face, n0:
// the 0-face's normal on the exterior side; n = 2 - alpha / pi (exterior
// angle n pi).  128 bytes.
struct alignas(16) Wedge {
    double a[3];
    double e[3];
    double t0[3];
    double n0[3];
    double len;     // edge length
    double n;
    int32_t face0, facen;
    int32_t mat0, matn;
};
static_assert(sizeof(Wedge) == 128, "wedge record size");

// Material constants derived on the host at the carrier frequency.
struct Mat {
    float eta_re, eta_im;      // complex relative permittivity eps_r - j sigma/(eps0 w)
    int32_t pec;               // perfect conductor
    float scat;                // scattering coefficient S: a reflection is diffuse with probability S^2
    double eta_re_d, eta_im_d; // the same in fp64
};

}  // namespace rt
