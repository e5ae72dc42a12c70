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

// Copies the first min(num_nodes, kLdsNodes) nodes into LDS (whole block).
__device__ __forceinline__ int stage_nodes(const DevScene& sc, Node* lds) {
    const int n = sc.num_nodes < kLdsNodes ? sc.num_nodes : kLdsNodes;
    const float4* src = reinterpret_cast<const float4*>(sc.nodes);
    float4* dst = reinterpret_cast<float4*>(lds);
    for (int i = threadIdx.x; i < 8 * n; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    return n;
}

// Slab test of one child box: entry distance (or +inf when missed).
__device__ __forceinline__ float slab(float lx, float hx, float ly, float hy, float lz, float hz, float ix, float iy,
                                      float iz, float oix, float oiy, float oiz, float tfar) {
    const float a0 = fmaf(lx, ix, -oix), a1 = fmaf(hx, ix, -oix);
    const float b0 = fmaf(ly, iy, -oiy), b1 = fmaf(hy, iy, -oiy);
    const float c0 = fmaf(lz, iz, -oiz), c1 = fmaf(hz, iz, -oiz);
    const float n = fmaxf(fmaxf(fminf(a0, a1), fminf(b0, b1)), fmaxf(fminf(c0, c1), 0.0f));
    const float f = fminf(fminf(fmaxf(a0, a1), fmaxf(b0, b1)), fminf(fmaxf(c0, c1), tfar));
    return n <= f * kWiden ? n : __builtin_inff();
}

__device__ __forceinline__ void cswap(float& ka, int& va, float& kb, int& vb) {
    if (kb < ka) {
        const float tk = ka;
        ka = kb;
        kb = tk;
        const int tv = va;
        va = vb;
        vb = tv;
    }
}

// Closest hit (ANY = false) or any hit on an open segment (ANY = true)
// through the 4-wide BVH.  Nodes with index < n_lds are read from the LDS
// copy, the others from global memory.  At an inner node the hit children
// are ordered by entry distance: the nearest is visited next, the others
// pushed farthest first.  OVF = false drops the private-memory continuation
// of the stack: only for trees whose worst-case stack need is <= kStack.
template <bool ANY, bool STATS = false, int BS = kBlock, bool OVF = true>
__device__ __forceinline__ int traverse(const DevScene& sc, const Node* lds_nodes, int n_lds, d3 o, d3 d, int excl0,
                                        int excl1, double tmin, double& tbest, int32_t (*stack)[BS],
                                        TravStats* ts = nullptr) {
    const int tid = threadIdx.x;
    const float ox = (float)o.x, oy = (float)o.y, oz = (float)o.z;
    const float ix = safe_inv(d.x), iy = safe_inv(d.y), iz = safe_inv(d.z);
    const float oix = ox * ix, oiy = oy * iy, oiz = oz * iz;
    float tfar = ANY ? kAnyFar : f_up(tbest);
    int best = -1;
    int node = 0, sp = 0;
    if constexpr (!OVF) {
        // Branch-free ordering: a hit child's key is its entry distance (>= 0,
        // so the float bits order as unsigned) with the slot in the two low
        // bits, a missed or empty child's key is ~0; four keys sort with
        // unsigned min/max.  Pushes write unconditionally and advance sp only
        // for hits (sp stays below the tree's stack need <= kStack), and the
        // top of the stack is read ahead at every step for the pop.
        while (true) {
            const int top = stack[sp > 0 ? sp - 1 : 0][tid];
            if (node >= 0) {
                if (STATS) ts->nodes++;
                float4 X0, X1, Y0, Y1, Z0, Z1;
                int4 ch;
                if (node < n_lds) {
                    const float4* np = reinterpret_cast<const float4*>(lds_nodes + node);
                    X0 = np[0]; X1 = np[1]; Y0 = np[2]; Y1 = np[3]; Z0 = np[4]; Z1 = np[5];
                    ch = reinterpret_cast<const int4*>(np)[6];
                    asm volatile("" ::: "memory");  // keeps these LDS reads apart from the global ones
                } else {
                    const float4* np = reinterpret_cast<const float4*>(sc.nodes + node);
                    X0 = np[0]; X1 = np[1]; Y0 = np[2]; Y1 = np[3]; Z0 = np[4]; Z1 = np[5];
                    ch = reinterpret_cast<const int4*>(np)[6];
                }
                if (STATS) ts->boxes += live_children(ch);
                const float k0 = slab(X0.x, X1.x, Y0.x, Y1.x, Z0.x, Z1.x, ix, iy, iz, oix, oiy, oiz, tfar);
                const float k1 = slab(X0.y, X1.y, Y0.y, Y1.y, Z0.y, Z1.y, ix, iy, iz, oix, oiy, oiz, tfar);
                const float k2 = slab(X0.z, X1.z, Y0.z, Y1.z, Z0.z, Z1.z, ix, iy, iz, oix, oiy, oiz, tfar);
                const float k3 = slab(X0.w, X1.w, Y0.w, Y1.w, Z0.w, Z1.w, ix, iy, iz, oix, oiy, oiz, tfar);
                auto key = [](float k, int c, uint32_t slot) {
                    return (k < __builtin_inff() && c != kEmptyChild) ? ((__float_as_uint(k) & ~3u) | slot) : ~0u;
                };
                uint32_t q0 = key(k0, ch.x, 0u), q1 = key(k1, ch.y, 1u), q2 = key(k2, ch.z, 2u),
                         q3 = key(k3, ch.w, 3u);
                int c0 = ch.x, c1 = ch.y, c2 = ch.z, c3 = ch.w;
                // compare-exchange of (key, child) pairs as selects (no branches)
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
                stack[sp][tid] = c3;
                sp += q3 != ~0u;
                stack[sp][tid] = c2;
                sp += q2 != ~0u;
                stack[sp][tid] = c1;
                sp += q1 != ~0u;
                if (q0 != ~0u) {
                    node = c0;
                } else {  // no child hit, so nothing was pushed: top is still the top
                    if (sp == 0) break;
                    node = top;
                    --sp;
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
                node = top;
                --sp;
            }
        }
        return best;
    }
    int32_t ovf[OVF ? kStackOverflow : 1];  // entries beyond the LDS stack (deep trees only)
    auto push = [&](int v) {
        if (!OVF || sp < kStack) stack[sp][tid] = v;
        else ovf[sp - kStack] = v;
        ++sp;
    };
    auto pop = [&]() {
        --sp;
        int v;
        if (!OVF || sp < kStack) {
            v = stack[sp][tid];
            asm volatile("" ::: "memory");  // an LDS read, not a flat one shared with ovf
        } else {
            v = ovf[sp - kStack];
        }
        return v;
    };
    while (true) {
        if (node >= 0) {
            if (STATS) ts->nodes++;
            float4 X0, X1, Y0, Y1, Z0, Z1;
            int4 ch;
            if (node < n_lds) {
                const float4* np = reinterpret_cast<const float4*>(lds_nodes + node);
                X0 = np[0]; X1 = np[1]; Y0 = np[2]; Y1 = np[3]; Z0 = np[4]; Z1 = np[5];
                ch = reinterpret_cast<const int4*>(np)[6];
                // keeps the two branches distinct, so that the LDS reads are not
                // merged with the global ones into generic (flat) loads
                asm volatile("" ::: "memory");
            } else {
                const float4* np = reinterpret_cast<const float4*>(sc.nodes + node);
                X0 = np[0]; X1 = np[1]; Y0 = np[2]; Y1 = np[3]; Z0 = np[4]; Z1 = np[5];
                ch = reinterpret_cast<const int4*>(np)[6];
            }
            if (STATS) ts->boxes += live_children(ch);
            float k0 = slab(X0.x, X1.x, Y0.x, Y1.x, Z0.x, Z1.x, ix, iy, iz, oix, oiy, oiz, tfar);
            float k1 = slab(X0.y, X1.y, Y0.y, Y1.y, Z0.y, Z1.y, ix, iy, iz, oix, oiy, oiz, tfar);
            float k2 = slab(X0.z, X1.z, Y0.z, Y1.z, Z0.z, Z1.z, ix, iy, iz, oix, oiy, oiz, tfar);
            float k3 = slab(X0.w, X1.w, Y0.w, Y1.w, Z0.w, Z1.w, ix, iy, iz, oix, oiy, oiz, tfar);
            int c0 = ch.x, c1 = ch.y, c2 = ch.z, c3 = ch.w;
            if (c1 == kEmptyChild) k1 = __builtin_inff();
            if (c2 == kEmptyChild) k2 = __builtin_inff();
            if (c3 == kEmptyChild) k3 = __builtin_inff();
            // sorting network on (entry distance, child)
            cswap(k0, c0, k1, c1);
            cswap(k2, c2, k3, c3);
            cswap(k0, c0, k2, c2);
            cswap(k1, c1, k3, c3);
            cswap(k1, c1, k2, c2);
            if (k3 < __builtin_inff()) push(c3);
            if (k2 < __builtin_inff()) push(c2);
            if (k1 < __builtin_inff()) push(c1);
            if (k0 < __builtin_inff()) {
                node = c0;
            } else {
                if (sp == 0) break;
                node = pop();
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
            node = pop();
        }
    }
    return best;
}

}  // namespace rt
