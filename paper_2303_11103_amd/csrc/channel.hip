// Channel responses from paths for gfx950 (paper Sec. II-A: paths become
// channel impulse responses, with synthetic arrays and Doppler; Sec. III-A:
// channel frequency responses of an OFDM system with 128 subcarriers spaced
// 30 kHz apart).
//
// A path p has a coefficient a_p (without the delay phase), a delay tau_p and
// unit vectors k_t (departure, from the angles of departure) and k_r (from the
// receiver towards the arriving wave, from the angles of arrival).  With the
// e^{+j w t} convention, an array element at offset r from the array centre
// sees a plane wave earlier by (k . r) / c (synthetic array, plane-wave
// assumption at the carrier wavelength), and moving devices shift the path's
// frequency by f_D = (v_tx . k_t + v_rx . k_r) / lambda.  The response at time
// step n (t = n / fs), receive element j, transmit element i and subcarrier k
// (baseband frequency f_k = (k - floor(K/2)) spacing) is
//   H = sum_p a_p exp(j 2 pi phi_p),
//   phi_p = -(f_c + f_k) tau_p + (k_t . r_i + k_r . r_j) / lambda + f_D t,
// the phase in cycles evaluated in fp64 and reduced modulo 1 before the sine.
#include "kernels.h"

namespace rt {
namespace {

__device__ __forceinline__ d3 unit_of(float th, float ph) {
    double st, ct, sp, cp;
    sincos((double)th, &st, &ct);
    sincos((double)ph, &sp, &cp);
    return d3{st * cp, st * sp, ct};
}

// Phase (cycles) of path p at output index (t, j, i, k).
__device__ __forceinline__ double path_phase(const CfrArgs& c, int64_t pair, int p, int t, int j, int i, int k) {
    const int64_t slot = pair * c.P + p;
    const d3 kt = unit_of(c.aod[2 * slot], c.aod[2 * slot + 1]);
    const d3 kr = unit_of(c.aoa[2 * slot], c.aoa[2 * slot + 1]);
    const int tx = (int)(pair / c.nrx), rx = (int)(pair % c.nrx);
    const double* ri = c.tx_el + 3 * i;
    const double* rj = c.rx_el + 3 * j;
    const double* vt = c.v_tx + 3 * tx;
    const double* vr = c.v_rx + 3 * rx;
    const double arr = (kt.x * ri[0] + kt.y * ri[1] + kt.z * ri[2] + kr.x * rj[0] + kr.y * rj[1] + kr.z * rj[2]) /
                       c.lambda;
    const double fd = (kt.x * vt[0] + kt.y * vt[1] + kt.z * vt[2] + kr.x * vr[0] + kr.y * vr[1] + kr.z * vr[2]) /
                      c.lambda;
    const double fk = (double)(k - c.K / 2) * c.spacing;
    double ph = -(c.freq + fk) * (double)c.tau[slot] + arr + fd * ((double)t / c.fs);
    return ph - floor(ph);
}

__device__ __forceinline__ void out_index(const CfrArgs& c, int64_t o, int64_t& pair, int& t, int& j, int& i, int& k) {
    k = (int)(o % c.K);
    o /= c.K;
    i = (int)(o % c.nt_el);
    o /= c.nt_el;
    j = (int)(o % c.nr_el);
    o /= c.nr_el;
    t = (int)(o % c.T);
    pair = o / c.T;
}

// One thread per output entry: sum over the pair's paths.
__global__ void cfr_kernel(CfrArgs c) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= c.total) return;
    int64_t pair;
    int t, j, i, k;
    out_index(c, o, pair, t, j, i, k);
    double re = 0.0, im = 0.0;
    for (int p = 0; p < c.P; ++p) {
        const int64_t slot = pair * c.P + p;
        if (c.depth[slot] < 0) continue;
        double s, co;
        sincospi(2.0 * path_phase(c, pair, p, t, j, i, k), &s, &co);
        const double ar = c.a[2 * slot], ai = c.a[2 * slot + 1];
        re += ar * co - ai * s;
        im += ar * s + ai * co;
    }
    c.H[2 * o] = (float)re;
    c.H[2 * o + 1] = (float)im;
}

// Adjoint of the linear map a -> H: g_p = sum over the pair's outputs of
// conj(G) exp(j 2 pi phi_p), one thread per path slot.
__global__ void cfr_adjoint_kernel(CfrArgs c, const float* __restrict__ G, double* __restrict__ g) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= c.npairs * c.P) return;
    const int64_t pair = slot / c.P;
    const int p = (int)(slot % c.P);
    double re = 0.0, im = 0.0;
    if (c.depth[slot] >= 0) {
        const int64_t per = (int64_t)c.T * c.nr_el * c.nt_el * c.K;
        for (int64_t q = 0; q < per; ++q) {
            const int64_t o = pair * per + q;
            int64_t pr;
            int t, j, i, k;
            out_index(c, o, pr, t, j, i, k);
            double s, co;
            sincospi(2.0 * path_phase(c, pair, p, t, j, i, k), &s, &co);
            const double gr = G[2 * o], gi = -G[2 * o + 1];  // conj(G)
            re += gr * co - gi * s;
            im += gr * s + gi * co;
        }
    }
    g[2 * slot] = re;
    g[2 * slot + 1] = im;
}

}  // namespace

hipError_t launch_cfr(const CfrArgs& c, hipStream_t s) {
    if (c.total <= 0) return hipSuccess;
    hipLaunchKernelGGL(cfr_kernel, dim3((unsigned)((c.total + 255) / 256)), dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_cfr_adjoint(const CfrArgs& c, const float* G, double* g, hipStream_t s) {
    const int64_t n = c.npairs * c.P;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(cfr_adjoint_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, c, G, g);
    return hipGetLastError();
}

}  // namespace rt
