// BVH traversal shared by the shoot-and-bounce, image-method and gradient
// kernels: fp32 conservative slab tests on a binary BVH (both child boxes per
// node) with a per-lane stack in LDS, fp64 Moller-Trumbore on triangles
// (double sided, inclusive edges, a triangle of an excluded face is skipped).
#pragma once
#include "kernels.h"

namespace rt {

constexpr int kBlock = 256;       // block size of kernels that do not stage nodes
constexpr int kTraceBlock = 512;  // block size of the shoot-and-bounce kernels
constexpr int kStack = kMaxDepth + 2;
constexpr int kLdsNodes = 256;    // top BVH nodes (breadth-first order) staged in LDS
constexpr float kDn = 1.0f - 1e-6f;  // conservative slab interval factors
constexpr float kUp = 1.0f + 1e-6f;

// Smallest float >= t for t >= 0 (inf stays inf).
__device__ __forceinline__ float f_up(double t) {
    float f = (float)t;
    if ((double)f < t) f = __uint_as_float(__float_as_uint(f) + 1u);
    return f;
}

__device__ __forceinline__ float safe_inv(double v) {
    float f = fabs(v) > 1e-20 ? (float)v : copysignf(1e-20f, (float)v);
    return 1.0f / f;
}

// Moller-Trumbore in fp64 without the division: returns true and updates
// (best, tbest) when triangle k is hit at tmin < t < tbest.
__device__ __forceinline__ bool tri_test(const Tri* __restrict__ tris, int k, d3 o, d3 d, int excl0, int excl1,
                                         double tmin, double& tbest, bool segment_mode) {
    const Tri* tp = tris + k;
    const int4 meta = *reinterpret_cast<const int4*>(reinterpret_cast<const char*>(tp) + 80);
    if (meta.x == excl0 || meta.x == excl1) return false;
    const double2* q = reinterpret_cast<const double2*>(tp);
    const double2 q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4];
    const d3 v0{q0.x, q0.y, q1.x}, e1{q1.y, q2.x, q2.y}, e2{q3.x, q3.y, q4.x};
    const double thr = q4.y;
    const d3 P = cross(d, e2);
    double det = dot(e1, P);
    if (fabs(det) < thr) return false;
    const d3 T = sub(o, v0);
    double un = dot(T, P);
    const d3 Q = cross(T, e1);
    double vn = dot(d, Q);
    double tn = dot(e2, Q);
    if (det < 0.0) {
        det = -det;
        un = -un;
        vn = -vn;
        tn = -tn;
    }
    if (!(un >= 0.0 && vn >= 0.0 && un + vn <= det)) return false;
    if (segment_mode) {  // open segment (tmin, 1 - tmin) in units of |d|
        double t = tn / det;
        return t > tmin && t < 1.0 - tmin;
    }
    if (!(tn > tmin * det && tn < tbest * det)) return false;
    double t = tn / det;
    if (!(t > tmin && t < tbest)) return false;
    tbest = t;
    return true;
}

// Closest hit (ANY = false) or any hit on an open segment (ANY = true).
// Work counters of one traversal (inner nodes visited, triangles tested).
struct TravStats {
    uint32_t nodes = 0;
    uint32_t tris = 0;
};

// Copies the first min(num_nodes, kLdsNodes) nodes into LDS (whole block).
__device__ __forceinline__ int stage_nodes(const DevScene& sc, Node* lds) {
    const int n = sc.num_nodes < kLdsNodes ? sc.num_nodes : kLdsNodes;
    const float4* src = reinterpret_cast<const float4*>(sc.nodes);
    float4* dst = reinterpret_cast<float4*>(lds);
    for (int i = threadIdx.x; i < 4 * n; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    return n;
}

// Nodes with index < n_lds are read from the LDS copy, the others from
// global memory (L2-resident for the scenes here).
template <bool ANY, bool STATS = false, int BS = kBlock>
__device__ __forceinline__ int traverse(const DevScene& sc, const Node* lds_nodes, int n_lds, d3 o, d3 d, int excl0,
                                        int excl1, double tmin, double& tbest, int32_t (*stack)[BS],
                                        TravStats* ts = nullptr) {
    const int tid = threadIdx.x;
    const float ox = (float)o.x, oy = (float)o.y, oz = (float)o.z;
    const float ix = safe_inv(d.x), iy = safe_inv(d.y), iz = safe_inv(d.z);
    const float oix = ox * ix, oiy = oy * iy, oiz = oz * iz;
    float tfar = ANY ? kUp : f_up(tbest);
    int best = -1;
    int node = 0, sp = 0;
    while (true) {
        if (node >= 0) {
            if (STATS) ts->nodes++;
            float4 A, B, C;
            int4 ch;
            if (node < n_lds) {
                const float4* np = reinterpret_cast<const float4*>(lds_nodes + node);
                A = np[0];
                B = np[1];
                C = np[2];
                ch = reinterpret_cast<const int4*>(np)[3];
            } else {
                const float4* np = reinterpret_cast<const float4*>(sc.nodes + node);
                A = np[0];
                B = np[1];
                C = np[2];
                ch = reinterpret_cast<const int4*>(np)[3];
            }
            float a0 = fmaf(A.x, ix, -oix), a1 = fmaf(A.y, ix, -oix);
            float b0 = fmaf(A.z, iy, -oiy), b1 = fmaf(A.w, iy, -oiy);
            float c0 = fmaf(C.x, iz, -oiz), c1 = fmaf(C.y, iz, -oiz);
            float n0 = fmaxf(fmaxf(fminf(a0, a1), fminf(b0, b1)), fmaxf(fminf(c0, c1), 0.0f));
            float f0 = fminf(fminf(fmaxf(a0, a1), fmaxf(b0, b1)), fminf(fmaxf(c0, c1), tfar));
            float a2 = fmaf(B.x, ix, -oix), a3 = fmaf(B.y, ix, -oix);
            float b2 = fmaf(B.z, iy, -oiy), b3 = fmaf(B.w, iy, -oiy);
            float c2 = fmaf(C.z, iz, -oiz), c3 = fmaf(C.w, iz, -oiz);
            float n1 = fmaxf(fmaxf(fminf(a2, a3), fminf(b2, b3)), fmaxf(fminf(c2, c3), 0.0f));
            float f1 = fminf(fminf(fmaxf(a2, a3), fmaxf(b2, b3)), fminf(fmaxf(c2, c3), tfar));
            bool h0 = n0 * kDn <= f0 * kUp;
            bool h1 = n1 * kDn <= f1 * kUp;
            if (h0 && h1) {
                bool first0 = n0 <= n1;
                stack[sp++][tid] = first0 ? ch.y : ch.x;
                node = first0 ? ch.x : ch.y;
            } else if (h0) {
                node = ch.x;
            } else if (h1) {
                node = ch.y;
            } else {
                if (sp == 0) break;
                node = stack[--sp][tid];
            }
        } else {
            const int code = ~node;
            const int first = code >> kLeafShift, cnt = (code & (kMaxLeaf - 1)) + 1;
            if (STATS) ts->tris += cnt;
            for (int k = first; k < first + cnt; ++k) {
                if (tri_test(sc.tris, k, o, d, excl0, excl1, tmin, tbest, ANY)) {
                    best = k;
                    if (ANY) return best;
                    tfar = f_up(tbest);
                }
            }
            if (sp == 0) break;
            node = stack[--sp][tid];
        }
    }
    return best;
}

}  // namespace rt
