// Image-method kernels for gfx950 (paper Sec. II-B: for every candidate, an
// ordered list of scene primitives found by the shooting rays, the image
// method gives the specular path through the same primitives that ends
// exactly at the receiver; duplicates are removed, line of sight is added;
// Sec. II-A: paths are returned as coefficients and delays).
//
// Candidates are the distinct face sequences stored in the prefix table
// filled by the shoot-and-bounce kernels; one thread handles one
// (receiver, candidate) pair in fp64: images, back-traced reflection points,
// validity (segment parameter, front side, point inside the face), occlusion
// of every segment by an any-hit BVH traversal, then the field transfer
// through the Fresnel reflections and the receive pattern.
#include "traverse.h"

namespace rt {
namespace {

constexpr int kMaxK = 8;
constexpr double kC0 = 299792458.0;
constexpr double kOccEps = 1e-9;     // open-segment parameter range (eps, 1 - eps)
constexpr double kInFaceTol = 1e-9;  // [m]

__global__ void extract_candidates_kernel(const uint64_t* __restrict__ table, uint64_t cap, int32_t max_depth,
                                          Cand* __restrict__ out, uint32_t* count, uint32_t max_out) {
    uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= cap) return;
    uint64_t key = table[s];
    if (key == kEmptyKey) return;
    Cand c;
    int faces_rev[kMaxK];
    int k = 0;
    while (true) {
        faces_rev[k++] = (int32_t)(uint32_t)(key & 0xffffffffull);
        int64_t parent = (int64_t)(key >> 32) - 1;
        if (parent < 0 || k >= kMaxK) break;
        key = table[parent];
    }
    c.depth = k;
    for (int i = 0; i < kMaxK; ++i) c.faces[i] = i < k ? faces_rev[k - 1 - i] : -1;
    uint32_t at = atomicAdd(count, 1u);
    if (at < max_out) out[at] = c;
}

// Reception-sphere pairs: every (receiver, prefix slot) of the pair set
// becomes a candidate (face sequence rebuilt from the prefix table) tied to
// its receiver.
__global__ void extract_pairs_kernel(const uint64_t* __restrict__ pairs, uint64_t pairs_cap,
                                     const uint64_t* __restrict__ table, Cand* __restrict__ out,
                                     int32_t* __restrict__ out_rx, uint32_t* count, uint32_t max_out) {
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= pairs_cap) return;
    const uint64_t pk = pairs[s];
    if (pk == kEmptyKey) return;
    const int32_t r = (int32_t)(pk >> 32);
    const int32_t slot = (int32_t)(uint32_t)(pk & 0xffffffffull);
    int faces_rev[kMaxK];
    int k = 0;
    uint64_t key = table[slot];
    while (true) {
        faces_rev[k++] = (int32_t)(uint32_t)(key & 0xffffffffull);
        const int64_t parent = (int64_t)(key >> 32) - 1;
        if (parent < 0 || k >= kMaxK) break;
        key = table[parent];
    }
    Cand c;
    c.depth = k;
    for (int i = 0; i < kMaxK; ++i) c.faces[i] = i < k ? faces_rev[k - 1 - i] : -1;
    const uint32_t at = atomicAdd(count, 1u);
    if (at < max_out) {
        out[at] = c;
        out_rx[at] = r;
    }
}

__device__ __forceinline__ d3 ld3(const double* p) { return d3{p[0], p[1], p[2]}; }

__device__ __forceinline__ void sph_basis(d3 d, d3& th, d3& ph) {
    double rho = sqrt(d.x * d.x + d.y * d.y);
    double cp = 1.0, sp = 0.0;
    if (rho > 0.0) {
        cp = d.x / rho;
        sp = d.y / rho;
    }
    th = d3{d.z * cp, d.z * sp, -rho};
    ph = d3{-sp, cp, 0.0};
}

struct c3 {
    cd x, y, z;
};
__device__ __forceinline__ cd cdot(c3 a, d3 b) {
    return cd{a.x.re * b.x + a.y.re * b.y + a.z.re * b.z, a.x.im * b.x + a.y.im * b.y + a.z.im * b.z};
}
__device__ __forceinline__ c3 reflect_field(c3 E, d3 ep, d3 eli, d3 elr, cd rp, cd rl) {
    cd ap = cmul(rp, cdot(E, ep)), al = cmul(rl, cdot(E, eli));
    return c3{cadd(cmulr(ap, ep.x), cmulr(al, elr.x)), cadd(cmulr(ap, ep.y), cmulr(al, elr.y)),
              cadd(cmulr(ap, ep.z), cmulr(al, elr.z))};
}

__device__ bool in_face(const DevScene& sc, int f, d3 X) {
    const Face F = sc.faces[f];
    for (int i = 0; i < F.count; ++i) {
        const Tri t = sc.tris[sc.face_tris[F.first + i]];
        const d3 v0 = ld3(t.v0);
        const d3 e1 = ld3(t.e1), e2 = ld3(t.e2);
        const d3 v[3] = {v0, add(v0, e1), add(v0, e2)};
        d3 n = cross(e1, e2);
        n = scale(n, 1.0 / norm(n));
        bool ok = true;
        for (int j = 0; j < 3 && ok; ++j) {
            const d3 a = v[j], b = v[(j + 1) % 3];
            const d3 e = sub(b, a);
            const double dist = dot(cross(e, sub(X, a)), n) / norm(e);
            if (dist < -kInFaceTol) ok = false;
        }
        if (ok) return true;
    }
    return false;
}

__global__ __launch_bounds__(kBlock) void image_paths_kernel(PathArgs a, MatTable mats, int64_t max_items) {
    __shared__ int32_t stack[kStack][kBlock];
    __shared__ Node lds_nodes[kLdsNodes];
    const int n_lds = stage_nodes(a.sc, lds_nodes);
    const int64_t ncand = (int64_t)(*a.ncand);
    const int64_t per_rx = ncand + 1;
    // every candidate for every receiver, or (pair mode) the line of sight of
    // every receiver followed by the receiver-tied candidates
    const int64_t total = a.pair_rx ? a.nrx + ncand : per_rx * a.nrx;
    for (int64_t item = (int64_t)blockIdx.x * kBlock + threadIdx.x; item < total;
         item += (int64_t)gridDim.x * kBlock) {
        int r;
        int64_t c;
        if (a.pair_rx) {
            r = item < a.nrx ? (int)item : a.pair_rx[item - a.nrx];
            c = item < a.nrx ? -1 : item - a.nrx;
        } else {
            r = (int)(item / per_rx);
            c = item - (int64_t)r * per_rx - 1;
        }
        int K = 0;
        int fc[kMaxK];
        if (c >= 0) {
            const Cand cd_ = a.cands[c];
            K = cd_.depth;
            if (K > a.max_depth) continue;
            for (int i = 0; i < kMaxK; ++i) fc[i] = cd_.faces[i];
        }
        const d3 tx = d3{a.tx[0], a.tx[1], a.tx[2]};
        const d3 rx = ld3(a.rx + 3 * r);
        d3 I[kMaxK + 1];
        I[0] = tx;
        for (int k = 1; k <= K; ++k) {
            const Face F = a.sc.faces[fc[k - 1]];
            const d3 n = ld3(F.n), q = ld3(F.q);
            I[k] = sub(I[k - 1], scale(n, 2.0 * dot(sub(I[k - 1], q), n)));
        }
        d3 X[kMaxK + 2];
        X[0] = tx;
        X[K + 1] = rx;
        bool valid = true;
        for (int k = K; k >= 1 && valid; --k) {
            const Face F = a.sc.faces[fc[k - 1]];
            const d3 n = ld3(F.n), q = ld3(F.q);
            const d3 A = X[k + 1];
            const double den = dot(sub(I[k], A), n);
            if (den == 0.0) {
                valid = false;
                break;
            }
            const double t = dot(sub(q, A), n) / den;
            if (!(t > 0.0 && t < 1.0)) {
                valid = false;
                break;
            }
            X[k] = add(A, scale(sub(I[k], A), t));
        }
        for (int k = 1; k <= K && valid; ++k) {
            const Face F = a.sc.faces[fc[k - 1]];
            const d3 n = ld3(F.n), q = ld3(F.q);
            const double sp = dot(sub(X[k - 1], q), n), sn = dot(sub(X[k + 1], q), n);
            if (!(sp * sn > 0.0)) valid = false;
            else if (!in_face(a.sc, fc[k - 1], X[k])) valid = false;
        }
        for (int k = 0; k <= K && valid; ++k) {
            const int ea = k == 0 ? -1 : fc[k - 1];
            const int eb = k == K ? -1 : fc[k];
            double tb = 1.0;
            if (traverse<true>(a.sc, lds_nodes, n_lds, X[k], sub(X[k + 1], X[k]), ea, eb, kOccEps, tb, stack) >= 0)
                valid = false;
        }
        if (!valid) continue;
        // ---- coefficients
        d3 dir[kMaxK + 1];
        double L = 0.0;
        for (int k = 0; k <= K; ++k) {
            const d3 s = sub(X[k + 1], X[k]);
            const double l = norm(s);
            L += l;
            dir[k] = scale(s, 1.0 / l);
        }
        const d3 F0 = antenna_field(a.tx_ant, dir[0]);
        c3 E{cd{F0.x, 0}, cd{F0.y, 0}, cd{F0.z, 0}};
        d3 th0, ph0;
        sph_basis(dir[0], th0, ph0);
        c3 B0{cd{th0.x, 0}, cd{th0.y, 0}, cd{th0.z, 0}};
        c3 B1{cd{ph0.x, 0}, cd{ph0.y, 0}, cd{ph0.z, 0}};
        for (int k = 1; k <= K; ++k) {
            const Face F = a.sc.faces[fc[k - 1]];
            d3 n = ld3(F.n);
            const d3 din = dir[k - 1], dout = dir[k];
            if (dot(din, n) > 0.0) n = scale(n, -1.0);
            const double cos_i = -dot(din, n);
            cd rp, rl;
            fresnel(mats.m[F.mat], cos_i, rp, rl);
            const double share = specular_share(mats.m[F.mat]);
            rp = cmulr(rp, share);
            rl = cmulr(rl, share);
            const d3 ep = perp_basis(din, n);
            const d3 eli = cross(ep, din), elr = cross(ep, dout);
            E = reflect_field(E, ep, eli, elr, rp, rl);
            B0 = reflect_field(B0, ep, eli, elr, rp, rl);
            B1 = reflect_field(B1, ep, eli, elr, rp, rl);
        }
        const d3 dK = dir[K];
        d3 thK, phK;
        sph_basis(dK, thK, phK);
        const d3 mdK = scale(dK, -1.0);
        const d3 Fr = antenna_field(a.rx_ant[r], mdK);
        const cd pr = cdot(E, Fr);
        const double amp = a.lambda / (4.0 * kPi * L);
        const uint32_t slot = atomicAdd(a.counts + r, 1u);
        if (slot >= (uint32_t)a.P) continue;
        const int64_t at = (int64_t)r * a.P + slot;
        a.a[2 * at] = (float)(amp * pr.re);
        a.a[2 * at + 1] = (float)(amp * pr.im);
        const cd t00 = cdot(B0, thK), t01 = cdot(B1, thK), t10 = cdot(B0, phK), t11 = cdot(B1, phK);
        float* T = a.T + 8 * at;
        T[0] = (float)t00.re; T[1] = (float)t00.im;
        T[2] = (float)t01.re; T[3] = (float)t01.im;
        T[4] = (float)t10.re; T[5] = (float)t10.im;
        T[6] = (float)t11.re; T[7] = (float)t11.im;
        a.tau[at] = (float)(L / kC0);
        a.aod[2 * at] = (float)acos(fmin(fmax(dir[0].z, -1.0), 1.0));
        a.aod[2 * at + 1] = (float)atan2(dir[0].y, dir[0].x);
        a.aoa[2 * at] = (float)acos(fmin(fmax(mdK.z, -1.0), 1.0));
        a.aoa[2 * at + 1] = (float)atan2(mdK.y, mdK.x);
        a.depth[at] = K;
        for (int i = 0; i < a.fd; ++i) a.faces[(int64_t)a.fd * at + i] = i < K ? fc[i] : -1;
    }
}

// Order the paths of one receiver by (depth, faces) and write them to the
// caller's arrays; unused slots get a = 0, tau = -1, depth = -1, faces = -1.
__global__ void sort_paths_kernel(PathArgs a, int32_t nrx, float* a_out, float* T_out, float* tau_out, float* aod_out,
                                  float* aoa_out, int32_t* depth_out, int32_t* faces_out, int32_t* num_out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrx) return;
    const uint32_t cnt = a.counts[r];
    num_out[r] = (int32_t)cnt;
    const int n = (int)(cnt < (uint32_t)a.P ? cnt : (uint32_t)a.P);
    int order[256];
    for (int i = 0; i < n; ++i) order[i] = i;
    const int64_t base = (int64_t)r * a.P;
    auto less = [&](int x, int y) {
        const int dx = a.depth[base + x], dy = a.depth[base + y];
        if (dx != dy) return dx < dy;
        for (int i = 0; i < a.fd; ++i) {
            const int fx = a.faces[(base + x) * a.fd + i], fy = a.faces[(base + y) * a.fd + i];
            if (fx != fy) return fx < fy;
        }
        return false;
    };
    for (int i = 1; i < n; ++i) {
        int v = order[i], j = i - 1;
        while (j >= 0 && less(v, order[j])) {
            order[j + 1] = order[j];
            --j;
        }
        order[j + 1] = v;
    }
    for (int i = 0; i < a.P; ++i) {
        const int64_t o = base + i;
        if (i < n) {
            const int64_t s = base + order[i];
            a_out[2 * o] = a.a[2 * s];
            a_out[2 * o + 1] = a.a[2 * s + 1];
            for (int k = 0; k < 8; ++k) T_out[8 * o + k] = a.T[8 * s + k];
            tau_out[o] = a.tau[s];
            aod_out[2 * o] = a.aod[2 * s];
            aod_out[2 * o + 1] = a.aod[2 * s + 1];
            aoa_out[2 * o] = a.aoa[2 * s];
            aoa_out[2 * o + 1] = a.aoa[2 * s + 1];
            depth_out[o] = a.depth[s];
            for (int k = 0; k < a.fd; ++k) faces_out[o * a.fd + k] = a.faces[s * a.fd + k];
        } else {
            a_out[2 * o] = 0.0f;
            a_out[2 * o + 1] = 0.0f;
            for (int k = 0; k < 8; ++k) T_out[8 * o + k] = 0.0f;
            tau_out[o] = -1.0f;
            aod_out[2 * o] = aod_out[2 * o + 1] = 0.0f;
            aoa_out[2 * o] = aoa_out[2 * o + 1] = 0.0f;
            depth_out[o] = -1;
            for (int k = 0; k < a.fd; ++k) faces_out[o * a.fd + k] = -1;
        }
    }
}

// P[r] = sum over the valid slots of |a|^2 (fp64 accumulation of the fp32 a).
__global__ void paths_power_kernel(const float* __restrict__ a, const int32_t* __restrict__ depth, int64_t n, int P,
                                   double* __restrict__ power) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double acc = 0.0;
    for (int j = 0; j < P; ++j) {
        const int64_t at = r * P + j;
        if (depth[at] < 0) continue;
        const double re = a[2 * at], im = a[2 * at + 1];
        acc += re * re + im * im;
    }
    power[r] = acc;
}

}  // namespace

hipError_t launch_paths_power(const float* a, const int32_t* depth, int64_t n, int P, double* power, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(paths_power_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, depth, n, P, power);
    return hipGetLastError();
}

hipError_t launch_extract_candidates(const uint64_t* table, uint64_t cap, int32_t max_depth, Cand* out,
                                     uint32_t* count, uint32_t max_out, hipStream_t s) {
    const uint64_t blocks = (cap + 255) / 256;
    hipLaunchKernelGGL(extract_candidates_kernel, dim3((unsigned)blocks), dim3(256), 0, s, table, cap, max_depth,
                       out, count, max_out);
    return hipGetLastError();
}

hipError_t launch_extract_pairs(const uint64_t* pairs, uint64_t pairs_cap, const uint64_t* table, Cand* out,
                                int32_t* out_rx, uint32_t* count, uint32_t max_out, hipStream_t s) {
    const uint64_t blocks = (pairs_cap + 255) / 256;
    hipLaunchKernelGGL(extract_pairs_kernel, dim3((unsigned)blocks), dim3(256), 0, s, pairs, pairs_cap, table, out,
                       out_rx, count, max_out);
    return hipGetLastError();
}

hipError_t launch_image_paths(const PathArgs& a, const MatTable& mats, int64_t max_items, hipStream_t s) {
    int64_t blocks = (max_items + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(image_paths_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, a, mats, max_items);
    return hipGetLastError();
}

hipError_t launch_sort_paths(const PathArgs& a, int32_t nrx, float* a_out, float* T_out, float* tau_out,
                             float* aod_out, float* aoa_out, int32_t* depth_out, int32_t* faces_out,
                             int32_t* num_paths_out, hipStream_t s) {
    const int blocks = (nrx + 63) / 64;
    hipLaunchKernelGGL(sort_paths_kernel, dim3(blocks), dim3(64), 0, s, a, nrx, a_out, T_out, tau_out, aod_out,
                       aoa_out, depth_out, faces_out, num_paths_out);
    return hipGetLastError();
}

}  // namespace rt
