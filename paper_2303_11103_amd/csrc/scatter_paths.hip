// Diffusely scattered paths for gfx950 (paper Sec. II-B lists diffuse
// reflection among the interactions of the tracer; Sec. II-A lets paths be
// computed with scattering).  The Lambertian model of the coverage maps (a
// fraction S^2 of the reflected power leaves diffusely with the intensity
// pattern cos / pi) becomes paths through the ray tubes of the lattice: every
// hit of a specularly traced ray is a scattering point of solid angle 4 pi / N
// for every receiver in front of its face that sees it, with
//   a = lambda / (4 pi) S w sqrt((4 pi / N) cos_s / pi) / r_s F_rx(-k) . E_s,
// E_s the reflected components (r_perp a_perp, r_par a_par) of the ray's field
// on the transverse basis of the scattered direction k, and w the product of
// sqrt(1 - S^2) over the earlier (specular) reflections.
//
// Per chunk of lattice rays, four passes:
//   1. points: one thread per ray traces max_depth segments (closest hit,
//      fp64) and writes one record per hit, [ray][depth], holding the point,
//      the normal facing the ray, the ray length, the face and the 2x2
//      complex map G from the departure components (theta, phi) of the field
//      to the scattered components (perp, par), S w and the Fresnel
//      coefficients included;
//   2. visibility: one thread per (receiver, record): front side of the face
//      and an any-hit traversal of the open segment point -> receiver; a wave
//      ballot stores 64 bits of the receiver's visibility mask;
//   3. scan: per receiver, the exclusive prefix of the mask popcounts;
//   4. write: one thread per visible (receiver, record) writes its path at
//      slot base + prefix + rank in the word, when below the capacity.
// Slots therefore follow (lattice ray, depth) for every receiver, with no
// sort and no atomics; the receiver's running base carries over the chunks.
#include "traverse.h"

namespace rt {
namespace {

constexpr double kC0s = 299792458.0;
constexpr double kOccEpsS = 1e-9;   // open-segment parameter range (eps, 1 - eps)

__device__ __forceinline__ d3 ldp(const double* p) { return d3{p[0], p[1], p[2]}; }

struct c3s {
    cd x, y, z;
};
__device__ __forceinline__ cd dotc(c3s a, d3 b) {
    return cd{a.x.re * b.x + a.y.re * b.y + a.z.re * b.z, a.x.im * b.x + a.y.im * b.y + a.z.im * b.z};
}
__device__ __forceinline__ c3s mk_real(d3 v) { return c3s{cd{v.x, 0.0}, cd{v.y, 0.0}, cd{v.z, 0.0}}; }
// r_perp (E . e_perp) e_perp + r_par (E . e_par_in) e_par_out
__device__ __forceinline__ c3s reflect_c3(c3s E, d3 ep, d3 eli, d3 elr, cd rp, cd rl) {
    const cd ap = cmul(rp, dotc(E, ep)), al = cmul(rl, dotc(E, eli));
    return c3s{cadd(cmulr(ap, ep.x), cmulr(al, elr.x)), cadd(cmulr(ap, ep.y), cmulr(al, elr.y)),
               cadd(cmulr(ap, ep.z), cmulr(al, elr.z))};
}
// unit vectors theta_hat, phi_hat of direction d (phi_hat = (0, 1, 0) on the axis)
__device__ __forceinline__ void sph_hat(d3 d, d3& th, d3& ph) {
    const double rho = sqrt(d.x * d.x + d.y * d.y);
    double cp = 1.0, sp = 0.0;
    if (rho > 0.0) {
        cp = d.x / rho;
        sp = d.y / rho;
    }
    th = d3{d.z * cp, d.z * sp, -rho};
    ph = d3{-sp, cp, 0.0};
}

__device__ __forceinline__ int64_t ray_index(const ScatArgs& a, int64_t j) {
    return a.begin + (a.pos0 + j) * a.stride;
}

__global__ __launch_bounds__(kBlock) void scatter_points_kernel(ScatArgs a, MatTable mats) {
    __shared__ int32_t stack[kStack][kBlock];
    __shared__ Node lds_nodes[kLdsNodes];
    const int n_lds = stage_nodes(a.sc, lds_nodes);
    const int D = a.max_depth;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.n; j += (int64_t)gridDim.x * blockDim.x) {
        d3 d = fib_dir(ray_index(a, j), a.num_rays);
        d3 o{a.tx[0], a.tx[1], a.tx[2]};
        d3 th, ph;
        sph_hat(d, th, ph);
        c3s U0 = mk_real(th), U1 = mk_real(ph);  // departure basis carried through the reflections
        double w = 1.0, s = 0.0;
        int excl = -1;
        bool alive = true;
        for (int k = 0; k < D; ++k) {
            ScatPoint* rec = a.points + j * D + k;
            int best = -1;
            double tbest = __builtin_inf();
            if (alive) best = traverse<false>(a.sc, lds_nodes, n_lds, o, d, excl, excl, a.tmin, tbest, stack);
            if (best < 0) {
                alive = false;
                rec->face = -1;
                rec->scat = 0;
                continue;
            }
            const Shade sh = a.sc.shades[best];
            d3 n{sh.n[0], sh.n[1], sh.n[2]};
            if (dot(d, n) > 0.0) n = scale(n, -1.0);
            const double cos_i = -dot(d, n);
            const d3 p = add(o, scale(d, tbest));
            s += tbest;
            cd rp, rl;
            fresnel(mats.m[sh.mat], cos_i, rp, rl);
            const d3 ep = perp_basis(d, n);
            const d3 eli = cross(ep, d);
            const d3 dr = add(d, scale(n, 2.0 * cos_i));
            const d3 elr = cross(ep, dr);
            const double S = (double)mats.m[sh.mat].scat;
            rec->p[0] = p.x;
            rec->p[1] = p.y;
            rec->p[2] = p.z;
            rec->n[0] = n.x;
            rec->n[1] = n.y;
            rec->n[2] = n.z;
            rec->s = s;
            rec->face = sh.face;
            rec->scat = S > 0.0 ? 1 : 0;
            if (S > 0.0) {
                const double sw = S * w;
                const cd g00 = cmulr(cmul(rp, dotc(U0, ep)), sw), g01 = cmulr(cmul(rp, dotc(U1, ep)), sw);
                const cd g10 = cmulr(cmul(rl, dotc(U0, eli)), sw), g11 = cmulr(cmul(rl, dotc(U1, eli)), sw);
                rec->g[0] = g00.re;
                rec->g[1] = g00.im;
                rec->g[2] = g01.re;
                rec->g[3] = g01.im;
                rec->g[4] = g10.re;
                rec->g[5] = g10.im;
                rec->g[6] = g11.re;
                rec->g[7] = g11.im;
            }
            U0 = reflect_c3(U0, ep, eli, elr, rp, rl);
            U1 = reflect_c3(U1, ep, eli, elr, rp, rl);
            w *= sqrt(1.0 - S * S);
            o = p;
            d = dr;
            excl = sh.face;
        }
    }
}

// One thread per (receiver, record); nrec_pad is a multiple of 64, so a wave
// covers 64 consecutive records of one receiver and its ballot is one mask word.
__global__ __launch_bounds__(kBlock) void scatter_visibility_kernel(ScatArgs a) {
    __shared__ int32_t stack[kStack][kBlock];
    __shared__ Node lds_nodes[kLdsNodes];
    const int n_lds = stage_nodes(a.sc, lds_nodes);
    const int64_t nrec = a.n * a.max_depth;
    const int64_t total = (int64_t)a.nrx * a.nrec_pad;
    for (int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; item < total;
         item += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = item / a.nrec_pad;
        const int64_t q = item - r * a.nrec_pad;
        bool vis = false;
        if (q < nrec) {
            const ScatPoint* rec = a.points + q;
            if (rec->scat) {
                const d3 p = ldp(rec->p), n = ldp(rec->n);
                const d3 R{a.rx[3 * r], a.rx[3 * r + 1], a.rx[3 * r + 2]};
                const d3 v = sub(R, p);
                if (dot(v, n) > 0.0) {
                    double tb = 1.0;
                    vis = traverse<true>(a.sc, lds_nodes, n_lds, p, v, rec->face, -1, kOccEpsS, tb, stack) < 0;
                }
            }
        }
        const uint64_t m = __ballot(vis);
        if ((threadIdx.x & 63) == 0) a.masks[item >> 6] = m;
    }
}

// Per receiver (one block each, grid-stride over receivers): prefix[r][w] =
// number of visible records of the receiver in mask words 0..w-1 of this
// chunk; chunk_total[r] = all of them.
constexpr int kScanBlock = 256;
__global__ __launch_bounds__(kScanBlock) void scatter_scan_kernel(const uint64_t* __restrict__ masks,
                                                                  uint32_t* __restrict__ prefix, int64_t nwords,
                                                                  int32_t nrx, int64_t* __restrict__ chunk_total) {
    __shared__ uint32_t wave_sum[kScanBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int r = blockIdx.x; r < nrx; r += gridDim.x) {
        const uint64_t* mr = masks + (int64_t)r * nwords;
        uint32_t* pr = prefix + (int64_t)r * nwords;
        uint32_t carry = 0;
        for (int64_t base = 0; base < nwords; base += kScanBlock) {
            const int64_t w = base + threadIdx.x;
            const uint32_t c = w < nwords ? (uint32_t)__popcll(mr[w]) : 0u;
            uint32_t incl = c;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t v = __shfl_up(incl, off);
                if (lane >= off) incl += v;
            }
            if (lane == 63) wave_sum[wv] = incl;
            __syncthreads();
            uint32_t before = carry;
            for (int i = 0; i < wv; ++i) before += wave_sum[i];
            if (w < nwords) pr[w] = before + incl - c;
            uint32_t tile = 0;
            for (int i = 0; i < kScanBlock / 64; ++i) tile += wave_sum[i];
            carry += tile;
            __syncthreads();
        }
        if (threadIdx.x == 0) chunk_total[r] = carry;
    }
}

__global__ __launch_bounds__(kBlock) void scatter_write_kernel(ScatArgs a) {
    const int64_t total = (int64_t)a.nrx * a.nrec_pad;
    const int D = a.max_depth;
    const double dom = 4.0 * kPi / (double)a.num_rays;
    for (int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; item < total;
         item += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t m = a.masks[item >> 6];
        const int lane = (int)(item & 63);
        if (!((m >> lane) & 1ull)) continue;
        const int64_t r = item / a.nrec_pad;
        const int64_t q = item - r * a.nrec_pad;
        const int64_t slot = a.base[r] + (int64_t)a.prefix[item >> 6] + __popcll(m & ((1ull << lane) - 1ull));
        if (slot >= a.P) continue;
        const ScatPoint rec = a.points[q];
        const int64_t j = q / D;
        const int k = (int)(q - j * D);
        const int64_t ray = ray_index(a, j);
        const d3 d0 = fib_dir(ray, a.num_rays);
        const d3 p = ldp(rec.p), n = ldp(rec.n);
        const d3 R{a.rx[3 * r], a.rx[3 * r + 1], a.rx[3 * r + 2]};
        const d3 v = sub(R, p);
        const double r_s = norm(v);
        const d3 ks = scale(v, 1.0 / r_s);
        const double cos_s = dot(ks, n);
        const double c = sqrt(dom * cos_s / kPi) / r_s;
        const d3 sp = perp_basis(ks, n);
        const d3 sl = cross(sp, ks);
        const cd g00{rec.g[0], rec.g[1]}, g01{rec.g[2], rec.g[3]}, g10{rec.g[4], rec.g[5]}, g11{rec.g[6], rec.g[7]};
        // scattered fields of the two departure basis vectors
        const c3s E0{cadd(cmulr(g00, sp.x), cmulr(g10, sl.x)), cadd(cmulr(g00, sp.y), cmulr(g10, sl.y)),
                     cadd(cmulr(g00, sp.z), cmulr(g10, sl.z))};
        const c3s E1{cadd(cmulr(g01, sp.x), cmulr(g11, sl.x)), cadd(cmulr(g01, sp.y), cmulr(g11, sl.y)),
                     cadd(cmulr(g01, sp.z), cmulr(g11, sl.z))};
        d3 th0, ph0, thk, phk;
        sph_hat(d0, th0, ph0);
        sph_hat(ks, thk, phk);
        const double L = rec.s + r_s;
        const d3 Ft = antenna_field(a.tx_ant, d0);
        const double ft = dot(Ft, th0), fp = dot(Ft, ph0);
        const d3 Fr = antenna_field(a.rx_ant[r], scale(ks, -1.0));
        const cd pr = cadd(cmulr(dotc(E0, Fr), ft), cmulr(dotc(E1, Fr), fp));
        const cd av = cmulr(pr, a.lambda / (4.0 * kPi) * c);
        const int64_t at = r * a.P + slot;
        a.a[2 * at] = (float)av.re;
        a.a[2 * at + 1] = (float)av.im;
        const double tsc = L * c;
        const cd t[4] = {dotc(E0, thk), dotc(E1, thk), dotc(E0, phk), dotc(E1, phk)};
        float* T = a.T + 8 * at;
        for (int i = 0; i < 4; ++i) {
            T[2 * i] = (float)(t[i].re * tsc);
            T[2 * i + 1] = (float)(t[i].im * tsc);
        }
        a.tau[at] = (float)(L / kC0s);
        a.aod[2 * at] = (float)acos(fmin(fmax(d0.z, -1.0), 1.0));
        a.aod[2 * at + 1] = (float)atan2(d0.y, d0.x);
        a.aoa[2 * at] = (float)acos(fmin(fmax(-ks.z, -1.0), 1.0));
        a.aoa[2 * at + 1] = (float)atan2(-ks.y, -ks.x);
        a.depth[at] = k + 1;
        a.ray[at] = ray;
        int32_t* fc = a.faces + at * a.fd;
        for (int i = 0; i < a.fd; ++i) fc[i] = i <= k ? a.points[j * D + i].face : -1;
    }
}

// base[r] += chunk_total[r]
__global__ void scatter_advance_kernel(int64_t* __restrict__ base, const int64_t* __restrict__ chunk_total,
                                       int32_t nrx) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrx) base[r] += chunk_total[r];
}

// Slots at or after min(count, P) of every receiver: a = T = 0, tau = -1,
// angles 0, depth = -1, ray = -1, faces = -1.
__global__ void scatter_tail_kernel(ScatArgs a) {
    const int64_t total = (int64_t)a.nrx * a.P;
    for (int64_t at = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; at < total;
         at += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = at / a.P;
        const int64_t slot = at - r * a.P;
        if (slot < a.base[r]) continue;
        a.a[2 * at] = 0.0f;
        a.a[2 * at + 1] = 0.0f;
        for (int i = 0; i < 8; ++i) a.T[8 * at + i] = 0.0f;
        a.tau[at] = -1.0f;
        a.aod[2 * at] = a.aod[2 * at + 1] = 0.0f;
        a.aoa[2 * at] = a.aoa[2 * at + 1] = 0.0f;
        a.depth[at] = -1;
        a.ray[at] = -1;
        for (int i = 0; i < a.fd; ++i) a.faces[at * a.fd + i] = -1;
    }
}

int64_t blocks_for(int64_t items, int64_t cap) {
    return std::max<int64_t>(1, std::min<int64_t>((items + kBlock - 1) / kBlock, cap));
}

}  // namespace

hipError_t launch_scatter_chunk(const ScatArgs& a, const MatTable& mats, hipStream_t s) {
    if (a.n <= 0 || a.max_depth <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_points_kernel, dim3((unsigned)blocks_for(a.n, 16384)), dim3(kBlock), 0, s, a, mats);
    const int64_t total = (int64_t)a.nrx * a.nrec_pad;
    hipLaunchKernelGGL(scatter_visibility_kernel, dim3((unsigned)blocks_for(total, 65536)), dim3(kBlock), 0, s, a);
    const int64_t nwords = a.nrec_pad / 64;
    hipLaunchKernelGGL(scatter_scan_kernel, dim3((unsigned)std::min<int64_t>(a.nrx, 65535)), dim3(kScanBlock), 0, s,
                       a.masks, a.prefix, nwords, a.nrx, a.chunk_total);
    hipLaunchKernelGGL(scatter_write_kernel, dim3((unsigned)blocks_for(total, 65536)), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(scatter_advance_kernel, dim3((unsigned)((a.nrx + 255) / 256)), dim3(256), 0, s, a.base,
                       a.chunk_total, a.nrx);
    return hipGetLastError();
}

hipError_t launch_scatter_tail(const ScatArgs& a, hipStream_t s) {
    const int64_t total = (int64_t)a.nrx * a.P;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_tail_kernel, dim3((unsigned)blocks_for(total, 65536)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace rt
