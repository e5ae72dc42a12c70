// BVH traversal shared by the shoot-and-bounce and image-method kernels: fp32
// conservative slab tests on a 4-wide BVH (the four child boxes of a node)
// with a per-lane stack in LDS, fp64 Moller-Trumbore on triangles (double
// sided, inclusive edges, a triangle of an excluded face is skipped).
#pragma once
#include "kernels.h"

namespace rt {

constexpr int kBlock = 256;       // block size of kernels that do not stage nodes
constexpr int kTraceBlock = 512;  // block size of the shoot-and-bounce kernels
constexpr int kStack = kStackEntries;
constexpr int kLdsNodes = 128;    // top BVH nodes (breadth-first order) staged in LDS, 16 KB
// Conservative slab interval: a box is entered when near <= far (1 + 3e-6).
// This accepts every box that near (1 - 1e-6) <= far (1 + 1e-6) accepts, each
// product rounded, at one multiplication per box.
constexpr float kWiden = 1.0f + 3e-6f;
constexpr float kAnyFar = 1.0f + 1e-6f;  // far limit of a segment query (t <= 1), slightly widened

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
    // every load of the record is issued before the first test that uses it
    const double2* q = reinterpret_cast<const double2*>(tp);
    const double2 q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4];
    const int4 meta = *reinterpret_cast<const int4*>(reinterpret_cast<const char*>(tp) + 80);
    const d3 v0{q0.x, q0.y, q1.x}, e1{q1.y, q2.x, q2.y}, e2{q3.x, q3.y, q4.x};
    const double thr = q4.y;
    // uses the vertex here, so that its load is not sunk below the determinant
    // test into a second round trip to memory
    asm volatile("" ::"v"(q0.x), "v"(q0.y), "v"(q1.x));
    const d3 P = cross(d, e2);
    double det = dot(e1, P);
    if (meta.x == excl0 || meta.x == excl1 || fabs(det) < thr) return false;
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
    uint32_t boxes = 0;  // child boxes of the visited nodes (empty slots not counted)
    uint32_t tris = 0;
};

__device__ __forceinline__ uint32_t live_children(int4 ch) {
    return (uint32_t)(ch.x != kEmptyChild) + (uint32_t)(ch.y != kEmptyChild) + (uint32_t)(ch.z != kEmptyChild) +
           (uint32_t)(ch.w != kEmptyChild);
}

// Copies the first min(num_nodes, kLdsNodes) nodes into LDS (whole block),
// in the global layout.
__device__ __forceinline__ int stage_nodes(const DevScene& sc, Node* lds) {
    const int n = sc.num_nodes < kLdsNodes ? sc.num_nodes : kLdsNodes;
    const float4* src = reinterpret_cast<const float4*>(sc.nodes);
    float4* dst = reinterpret_cast<float4*>(lds);
    for (int i = threadIdx.x; i < 8 * n; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    return n;
}

// Per-ray byte offsets of the near and far planes of each axis inside a node
// (lo at +0 and hi at +16 of the axis's 32-byte pair): a ray with a negative
// direction component enters a box through its hi plane.
struct Octant {
    uint32_t nx, ny, nz, fx, fy, fz;
};

__device__ __forceinline__ Octant ray_octant(float ix, float iy, float iz) {
    Octant q;
    q.nx = ix < 0.0f ? 16u : 0u;
    q.ny = iy < 0.0f ? 48u : 32u;
    q.nz = iz < 0.0f ? 80u : 64u;
    q.fx = q.nx ^ 16u;
    q.fy = q.ny ^ 16u;
    q.fz = q.nz ^ 16u;
    return q;
}

// Near and far planes of the four children (one float4 per plane, one lane
// per child) and the child references of the node at byte address p.
struct NodePlanes {
    float4 NX, NY, NZ, FX, FY, FZ;
    int4 ch;
};

// base: the node array (LDS or global); off: byte offset of the node (a
// multiple of 128, so the plane offsets can be or-ed in as 32-bit values);
// sw: the slot swizzle of the copy, (n & 7) * 16 in LDS, 0 in global memory.
__device__ __forceinline__ NodePlanes load_planes(const char* base, uint32_t off, uint32_t sw, const Octant& q) {
    NodePlanes n;
    n.NX = *reinterpret_cast<const float4*>(base + (off | (q.nx ^ sw)));
    n.FX = *reinterpret_cast<const float4*>(base + (off | (q.fx ^ sw)));
    n.NY = *reinterpret_cast<const float4*>(base + (off | (q.ny ^ sw)));
    n.FY = *reinterpret_cast<const float4*>(base + (off | (q.fy ^ sw)));
    n.NZ = *reinterpret_cast<const float4*>(base + (off | (q.nz ^ sw)));
    n.FZ = *reinterpret_cast<const float4*>(base + (off | (q.fz ^ sw)));
    n.ch = *reinterpret_cast<const int4*>(base + (off | (96u ^ sw)));
    return n;
}

// Sort key of one child box: its entry distance (>= 0, sign bit cleared so
// that -0 orders as 0; the float bits then order as unsigned) with the slot
// in the two low bits, or ~0 when the ray misses the box.  The planes come in
// ray order, so no per-axis min/max is needed; an empty slot (lo = +inf,
// hi = -inf on every axis) always misses.
__device__ __forceinline__ uint32_t box_key(float nx, float ny, float nz, float fx, float fy, float fz, float ix,
                                            float iy, float iz, float oix, float oiy, float oiz, float tfar,
                                            uint32_t slot) {
    const float tn = fmaxf(fmaxf(fmaf(nx, ix, -oix), fmaf(ny, iy, -oiy)), fmaxf(fmaf(nz, iz, -oiz), 0.0f));
    const float tf = fminf(fminf(fmaf(fx, ix, -oix), fmaf(fy, iy, -oiy)), fminf(fmaf(fz, iz, -oiz), tfar));
    return tn <= tf * kWiden ? ((__float_as_uint(tn) & 0x7ffffffcu) | slot) : ~0u;
}

// Closest hit (ANY = false) or any hit on an open segment (ANY = true)
// through the 4-wide BVH.  Nodes with index < n_lds are read from the LDS
// copy, the others from global memory.  At an inner node the hit children
// are ordered by entry distance: the nearest is visited next, the others
// pushed farthest first.  Leaves are parked and tested when the whole wave
// has one (see the loop).  OVF = false drops the private-memory continuation
// of the stack: only for trees whose worst-case stack need is <= kStack.
// STOP = true returns at the first hit closer than the tbest passed in (an
// occlusion test of the segment up to that distance).
template <bool ANY, bool STATS = false, int BS = kBlock, bool OVF = true, bool STOP = false>
__device__ __forceinline__ int traverse(const DevScene& sc, const Node* lds_nodes, int n_lds, d3 o, d3 d, int excl0,
                                        int excl1, double tmin, double& tbest, int32_t (*stack)[BS],
                                        TravStats* ts = nullptr) {
    const int tid = threadIdx.x;
    const float ox = (float)o.x, oy = (float)o.y, oz = (float)o.z;
    const float ix = safe_inv(d.x), iy = safe_inv(d.y), iz = safe_inv(d.z);
    const float oix = ox * ix, oiy = oy * iy, oiz = oz * iz;
    const Octant oct = ray_octant(ix, iy, iz);
    float tfar = ANY ? kAnyFar : f_up(tbest);
    int best = -1;
    int node = 0, sp = 0;
    int32_t ovf[OVF ? kStackOverflow : 1];  // entries beyond the LDS stack (deep trees only)
    // Pushes write unconditionally and advance sp only for hit children; the
    // top of the stack is read ahead at every step for the pop.
    auto put = [&](int at, int v) {
        if (!OVF || at < kStack) stack[at][tid] = v;
        else ovf[at - kStack] = v;
    };
    auto get = [&](int at) {
        int v;
        if (!OVF || at < kStack) {
            v = stack[at][tid];
            asm volatile("" ::: "memory");  // an LDS read, not a flat one shared with ovf
        } else {
            v = ovf[at - kStack];
        }
        return v;
    };
    // Leaves are postponed: a lane that reaches a leaf parks it and goes on
    // with its stack (speculatively, beside lanes still looking for a leaf);
    // the wave tests triangles only when no lane can make inner-node progress
    // without a pending leaf, so triangle tests run with most lanes active.
    constexpr int kDone = kEmptyChild;
    int leaf = 0;  // parked leaf code (negative), 0 = none
    // A leaf code leaves bits 23-30 all ones when the scene has at most 2^18
    // triangles; the references to leaves then carry the float exponent of
    // the leaf box's entry distance there, and a leaf taken off the stack or
    // parked is skipped when that exponent exceeds the one of the (widened)
    // closest hit: the box lies wholly beyond it.
    const uint32_t keep = sc.nt <= (1 << 18) ? 0x807FFFFFu : 0xFFFFFFFFu;
    const uint32_t dist_bits = ~keep;
    while (true) {
        const int top = get(sp > 0 ? sp - 1 : 0);
        const bool want_inner = node >= 0 && leaf == 0;
        if (__ballot(want_inner) != 0) {
            if (node >= 0) {
                if (STATS) ts->nodes++;
                NodePlanes np;
                const uint32_t off = (uint32_t)node * (uint32_t)sizeof(Node);
                if (node < n_lds) {
                    np = load_planes(reinterpret_cast<const char*>(lds_nodes), off, 0u, oct);
                    // keeps the two branches distinct, so that the LDS reads are not
                    // merged with the global ones into generic (flat) loads
                    asm volatile("" ::: "memory");
                } else {
                    np = load_planes(reinterpret_cast<const char*>(sc.nodes), off, 0u, oct);
                }
                if (STATS) ts->boxes += live_children(np.ch);
                uint32_t q0 = box_key(np.NX.x, np.NY.x, np.NZ.x, np.FX.x, np.FY.x, np.FZ.x, ix, iy, iz, oix, oiy, oiz,
                                      tfar, 0u);
                uint32_t q1 = box_key(np.NX.y, np.NY.y, np.NZ.y, np.FX.y, np.FY.y, np.FZ.y, ix, iy, iz, oix, oiy, oiz,
                                      tfar, 1u);
                uint32_t q2 = box_key(np.NX.z, np.NY.z, np.NZ.z, np.FX.z, np.FY.z, np.FZ.z, ix, iy, iz, oix, oiy, oiz,
                                      tfar, 2u);
                uint32_t q3 = box_key(np.NX.w, np.NY.w, np.NZ.w, np.FX.w, np.FY.w, np.FZ.w, ix, iy, iz, oix, oiy, oiz,
                                      tfar, 3u);
                int c0 = np.ch.x, c1 = np.ch.y, c2 = np.ch.z, c3 = np.ch.w;
                // sorting network of compare-exchanges on (key, child) as selects
                auto cx = [](uint32_t& a, int& ca, uint32_t& b, int& cb) {
                    const bool sw = b < a;
                    const uint32_t lo = sw ? b : a, hi = sw ? a : b;
                    const int clo = sw ? cb : ca, chi = sw ? ca : cb;
                    a = lo;
                    b = hi;
                    ca = clo;
                    cb = chi;
                };
                cx(q0, c0, q1, c1);
                cx(q2, c2, q3, c3);
                cx(q0, c0, q2, c2);
                cx(q1, c1, q3, c3);
                cx(q1, c1, q2, c2);
                // the entry distance's exponent into the leaf references (inner node
                // indices have zeros there and stay as they are)
                c0 = (int)((uint32_t)c0 & (q0 | keep));
                c1 = (int)((uint32_t)c1 & (q1 | keep));
                c2 = (int)((uint32_t)c2 & (q2 | keep));
                c3 = (int)((uint32_t)c3 & (q3 | keep));
                // a nearest child that is a leaf is parked at once when the lane
                // holds none; the next-nearest child is then visited next
                const bool park = q0 != ~0u && c0 < 0 && leaf == 0;
                if (park) leaf = c0;
                put(sp, c3);
                sp += q3 != ~0u;
                put(sp, c2);
                sp += q2 != ~0u;
                put(sp, c1);
                sp += (q1 != ~0u) & !park;
                const bool has_next = park ? q1 != ~0u : q0 != ~0u;
                if (has_next) {
                    node = park ? c1 : c0;
                } else if (sp == 0) {  // nothing pushed: top is still the top
                    node = kDone;
                } else {
                    node = top;
                    --sp;
                }
            } else if (node != kDone && leaf == 0) {
                leaf = node;
                if (sp == 0) {
                    node = kDone;
                } else {
                    node = top;
                    --sp;
                }
            }
        } else {
            if (leaf != 0) {
                if (((uint32_t)leaf & dist_bits) <= (__float_as_uint(tfar * kWiden) & 0x7F800000u)) {
                    const int code = ~(leaf | (int)dist_bits);
                    const int first = code >> kLeafShift, cnt = (code & (kMaxLeaf - 1)) + 1;
                    if (STATS) ts->tris += cnt;
                    for (int k = first; k < first + cnt; ++k) {
                        if (tri_test(sc.tris, k, o, d, excl0, excl1, tmin, tbest, ANY)) {
                            best = k;
                            if (ANY || STOP) return best;
                            tfar = f_up(tbest);
                        }
                    }
                }
                leaf = 0;
            }
            if (node < 0 && node != kDone) {
                leaf = node;
                if (sp == 0) {
                    node = kDone;
                } else {
                    node = top;
                    --sp;
                }
            }
            if (__ballot(leaf != 0 || node != kDone) == 0) break;
        }
    }
    return best;
}

}  // namespace rt
