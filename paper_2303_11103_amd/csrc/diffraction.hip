// First-order edge diffraction for gfx950 (paper Sec. II-B lists first-order
// diffraction among the interactions of the tracer).  One thread handles one
// (receiver, wedge) pair in fp64:
//   * diffraction point Q on the edge by Keller's law (equal angles of the
//     incident and diffracted rays with the edge), inside the edge;
//   * angles phi' (transmitter) and phi (receiver) about the edge, measured
//     from the 0-face through the exterior (0 < phi', phi < n pi);
//   * both legs unoccluded (any-hit traversals with the wedge faces skipped);
//   * uniform-theory (UTD) coefficients of a wedge with exterior angle n pi:
//       D_{s,h} = -e^{-j pi/4} / (2 n sqrt(2 pi k) sin b0) [
//           cot((pi + (phi - phi'))/2n) F(kL a+(phi - phi'))
//         + cot((pi - (phi - phi'))/2n) F(kL a-(phi - phi'))
//         + R0 cot((pi - (phi + phi'))/2n) F(kL a-(phi + phi'))
//         + Rn cot((pi + (phi + phi'))/2n) F(kL a+(phi + phi')) ]
//     with the Fresnel coefficients R0, Rn (perpendicular for D_s, parallel
//     for D_h) of the two faces at the local incidence cosines sin(b0)|sin phi'|
//     and sin(b0)|sin(n pi - phi)|, L = s' s sin^2 b0 / (s' + s);
//   * the vector field through the dyadic -b'b D_s - p'p D_h in the edge-fixed
//     unit vectors, spherical spreading sqrt(s' / (s (s + s'))).
// The transition function F(x) = 2j sqrt(x) e^{jx} int_sqrt(x)^inf e^{-j t^2} dt
// is evaluated from erfc(sqrt(x) e^{j pi/4}): the Maclaurin series of erf for
// x < 6 and Laplace's continued fraction of erfc (60 levels, evaluated from the
// tail) above; both are accurate to about 1e-14 there.
#include "traverse.h"

namespace rt {
namespace {

constexpr double kC0d = 299792458.0;
constexpr double kOccEpsD = 1e-9;

__device__ __forceinline__ d3 ldw(const double* p) { return d3{p[0], p[1], p[2]}; }
__device__ __forceinline__ cd cexpj(double t) { return cd{cos(t), sin(t)}; }

// F(x) for x >= 0.
__device__ cd transition(double x) {
    const double sx = sqrt(x);
    const cd z{sx * 0.70710678118654752440, sx * 0.70710678118654752440};  // sqrt(x) e^{j pi/4}
    if (x < 6.0) {
        // erf(z) = (2 z / sqrt(pi)) sum_n (-j x)^n / (n! (2n + 1)),  since z^2 = j x
        cd term{1.0, 0.0}, sum{0.0, 0.0};
        for (int n = 0; n < 80; ++n) {
            sum = cadd(sum, cmulr(term, 1.0 / (2 * n + 1)));
            term = cmulr(cmul(term, cd{0.0, -x}), 1.0 / (n + 1));
            if (fabs(term.re) + fabs(term.im) < 1e-18 * (fabs(sum.re) + fabs(sum.im))) break;
        }
        const cd erf = cmul(cmulr(z, 1.1283791670955126), sum);  // 2 / sqrt(pi)
        const cd erfc{1.0 - erf.re, -erf.im};
        // F = j sqrt(pi x) e^{j (x - pi/4)} erfc
        const cd ph = cexpj(x - 0.25 * kPi);
        return cmul(cd{0.0, sqrt(kPi * x)}, cmul(ph, erfc));
    }
    // erfc(z) = e^{-z^2} / sqrt(pi) K, K = 1/(z + (1/2)/(z + 1/(z + (3/2)/(z + ...)))),
    // so F = j sqrt(x) e^{-j pi/4} K (the e^{jx} of F cancels e^{-z^2} = e^{-jx})
    cd t = z;
    for (int m = 60; m >= 1; --m) t = cadd(z, cdiv(cd{0.5 * m, 0.0}, t));
    const cd K = cdiv(cd{1.0, 0.0}, t);
    return cmul(cd{0.0, sx}, cmul(cd{0.70710678118654752440, -0.70710678118654752440}, K));
}

// cot((pi + sign b)/(2n)) F(kL a^sign(b)); on a shadow boundary (infinite
// cotangent, vanishing F) the limit n sqrt(2 pi kL) sgn(eps) e^{j pi/4}.
__device__ cd utd_term(double kL, double n, double b, double sign) {
    const double arg = (kPi + sign * b) / (2.0 * n);
    const double N = rint((b + sign * kPi) / (2.0 * kPi * n));
    const double c = cos((2.0 * kPi * n * N - b) / 2.0);
    const double a = 2.0 * c * c;
    const double sn = sin(arg);
    if (fabs(sn) < 1e-12) {
        const double Nb = rint((kPi + sign * b) / (2.0 * kPi * n));
        const double eps = (kPi + sign * b) - 2.0 * kPi * n * Nb;
        const double m = n * sqrt(2.0 * kPi * kL) * (eps >= 0.0 ? 1.0 : -1.0);
        return cd{m * 0.70710678118654752440, m * 0.70710678118654752440};
    }
    return cmulr(transition(kL * a), cos(arg) / sn);
}

__device__ __forceinline__ double angle_about(const Wedge& w, d3 X, d3 Q) {
    const d3 u = sub(X, Q);
    double ph = atan2(dot(u, ldw(w.n0)), dot(u, ldw(w.t0)));
    if (ph < 0.0) ph += 2.0 * kPi;
    return ph;
}

__device__ __forceinline__ void face_fresnel(const MatTable& mats, int m, double cos_i, cd& rs, cd& rh) {
    fresnel(mats.m[m], cos_i, rs, rh);
}

// One diffracted path over wedge wi from S (antenna txa) to P (antenna rxa):
// false when there is none.  FULL also fills the transfer matrix and the
// directions; otherwise only the coefficient a.
struct DiffPath {
    cd a;
    cd T[4];
    double len;
    d3 s_in, s_out;
};

template <bool FULL>
__device__ bool diffracted(const DevScene& sc, const Node* lds_nodes, int n_lds, int32_t (*stack)[kBlock],
                           const MatTable& mats, double lambda, d3 S, const Antenna& txa, d3 P, const Antenna& rxa,
                           int wi, DiffPath& out) {
    const Wedge w = sc.wedges[wi];
    const d3 A = ldw(w.a), e = ldw(w.e);
    // Keller point: axial coordinates and distances from the edge line
    const double zs = dot(sub(S, A), e), zp = dot(sub(P, A), e);
    const double rs = norm(sub(sub(S, A), scale(e, zs))), rp = norm(sub(sub(P, A), scale(e, zp)));
    if (rs < 1e-9 || rp < 1e-9) return false;
    const double z = zs + (zp - zs) * rs / (rs + rp);
    if (!(z > 0.0 && z < w.len)) return false;
    const d3 Q = add(A, scale(e, z));
    const double phip = angle_about(w, S, Q), phi = angle_about(w, P, Q);
    const double lim = w.n * kPi;
    if (!(phip > 0.0 && phip < lim && phi > 0.0 && phi < lim)) return false;
    // both legs unoccluded (open segments, the two wedge faces skipped)
    double tb = 1.0;
    if (traverse<true>(sc, lds_nodes, n_lds, S, sub(Q, S), w.face0, w.facen, kOccEpsD, tb, stack) >= 0) return false;
    tb = 1.0;
    if (traverse<true>(sc, lds_nodes, n_lds, Q, sub(P, Q), w.face0, w.facen, kOccEpsD, tb, stack) >= 0) return false;
    // coefficients
    const double k = 2.0 * kPi / lambda;
    const d3 vin = sub(Q, S), vout = sub(P, Q);
    const double sp = norm(vin), s = norm(vout);
    const d3 sin_ = scale(vin, 1.0 / sp), sout = scale(vout, 1.0 / s);
    const double cb = fmin(fmax(dot(sin_, e), -1.0), 1.0);
    const double b0 = acos(cb);
    const double sb = sin(b0);
    const double L = sp * s * sb * sb / (sp + s);
    cd r0s, r0h, rns, rnh;
    face_fresnel(mats, w.mat0, sb * fabs(sin(phip)), r0s, r0h);
    face_fresnel(mats, w.matn, sb * fabs(sin(lim - phi)), rns, rnh);
    const double kL = k * L;
    const cd t1 = utd_term(kL, w.n, phi - phip, 1.0);
    const cd t2 = utd_term(kL, w.n, phi - phip, -1.0);
    const cd t3 = utd_term(kL, w.n, phi + phip, -1.0);
    const cd t4 = utd_term(kL, w.n, phi + phip, 1.0);
    // -e^{-j pi/4} / (2 n sqrt(2 pi k) sin b0)
    const double pm = -1.0 / (2.0 * w.n * sqrt(2.0 * kPi * k) * sb);
    const cd pre{pm * 0.70710678118654752440, -pm * 0.70710678118654752440};
    const cd t12 = cadd(t1, t2);
    const cd Ds = cmul(pre, cadd(t12, cadd(cmul(r0s, t3), cmul(rns, t4))));
    const cd Dh = cmul(pre, cadd(t12, cadd(cmul(r0h, t3), cmul(rnh, t4))));
    // edge-fixed unit vectors
    const d3 t0 = ldw(w.t0), n0 = ldw(w.n0);
    const d3 ph_in = add(scale(t0, -sin(phip)), scale(n0, cos(phip)));
    const d3 ph_out = add(scale(t0, -sin(phi)), scale(n0, cos(phi)));
    const d3 be_in = cross(ph_in, sin_), be_out = cross(ph_out, sout);
    // E_out = -Ds be_out (be_in . E) - Dh ph_out (ph_in . E); u . Dbar . v
    auto dyad = [&](d3 u, d3 v) {
        return csub(cmulr(Ds, -dot(u, be_out) * dot(be_in, v)), cmulr(Dh, dot(u, ph_out) * dot(ph_in, v)));
    };
    const double amp = 1.0 / sqrt(sp * s * (sp + s));
    const d3 Ft = antenna_field(txa, sin_);
    const d3 Fr = antenna_field(rxa, scale(sout, -1.0));
    out.a = cmulr(dyad(Fr, Ft), lambda / (4.0 * kPi) * amp);
    if (FULL) {
        // spherical unit vectors of s_in (departure) and s_out (direction of travel on arrival)
        auto basis = [](d3 d, d3& th, d3& ph) {
            const double rho = sqrt(d.x * d.x + d.y * d.y);
            double cp = 1.0, spn = 0.0;
            if (rho > 0.0) {
                cp = d.x / rho;
                spn = d.y / rho;
            }
            th = d3{d.z * cp, d.z * spn, -rho};
            ph = d3{-spn, cp, 0.0};
        };
        d3 thi, phi_i, tho, pho;
        basis(sin_, thi, phi_i);
        basis(sout, tho, pho);
        const double tsc = (sp + s) * amp;
        out.T[0] = cmulr(dyad(tho, thi), tsc);
        out.T[1] = cmulr(dyad(tho, phi_i), tsc);
        out.T[2] = cmulr(dyad(pho, thi), tsc);
        out.T[3] = cmulr(dyad(pho, phi_i), tsc);
        out.len = sp + s;
        out.s_in = sin_;
        out.s_out = sout;
    }
    return true;
}

__global__ __launch_bounds__(kBlock) void diffraction_kernel(PathArgs a, MatTable mats) {
    __shared__ int32_t stack[kStack][kBlock];
    __shared__ Node lds_nodes[kLdsNodes];
    const int n_lds = stage_nodes(a.sc, lds_nodes);
    const int64_t nw = a.sc.num_wedges;
    const int64_t total = (int64_t)a.nrx * nw;
    const d3 S{a.tx[0], a.tx[1], a.tx[2]};
    for (int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; item < total;
         item += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(item / nw);
        const int wi = (int)(item - (int64_t)r * nw);
        const d3 P{a.rx[3 * r], a.rx[3 * r + 1], a.rx[3 * r + 2]};
        DiffPath p;
        if (!diffracted<true>(a.sc, lds_nodes, n_lds, stack, mats, a.lambda, S, a.tx_ant, P, a.rx_ant[r], wi, p))
            continue;
        const uint32_t slot = atomicAdd(a.counts + r, 1u);
        if (slot >= (uint32_t)a.P) continue;
        const int64_t at = (int64_t)r * a.P + slot;
        a.a[2 * at] = (float)p.a.re;
        a.a[2 * at + 1] = (float)p.a.im;
        float* T = a.T + 8 * at;
        for (int i = 0; i < 4; ++i) {
            T[2 * i] = (float)p.T[i].re;
            T[2 * i + 1] = (float)p.T[i].im;
        }
        a.tau[at] = (float)(p.len / kC0d);
        a.aod[2 * at] = (float)acos(fmin(fmax(p.s_in.z, -1.0), 1.0));
        a.aod[2 * at + 1] = (float)atan2(p.s_in.y, p.s_in.x);
        a.aoa[2 * at] = (float)acos(fmin(fmax(-p.s_out.z, -1.0), 1.0));
        a.aoa[2 * at + 1] = (float)atan2(-p.s_out.y, -p.s_out.x);
        a.depth[at] = 1;
        a.faces[at] = wi;
    }
}

// Diffraction part of a coverage map: one thread per cell adds the path gain
// |a|^2 of every wedge's diffracted path to the cell centre (fixed wedge
// order, so the sum is deterministic).
__global__ __launch_bounds__(kBlock) void coverage_diffraction_kernel(DevScene sc, MatTable mats, double lambda,
                                                                      d3 S, Antenna txa, Antenna rxa, double gx0,
                                                                      double gy0, double gcell, double gz,
                                                                      int32_t gnx, int64_t cells,
                                                                      float* __restrict__ gain) {
    __shared__ int32_t stack[kStack][kBlock];
    __shared__ Node lds_nodes[kLdsNodes];
    const int n_lds = stage_nodes(sc, lds_nodes);
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t iy = c / gnx, ix = c - iy * gnx;
        const d3 P{gx0 + ((double)ix + 0.5) * gcell, gy0 + ((double)iy + 0.5) * gcell, gz};
        double acc = 0.0;
        for (int wi = 0; wi < sc.num_wedges; ++wi) {
            DiffPath p;
            if (diffracted<false>(sc, lds_nodes, n_lds, stack, mats, lambda, S, txa, P, rxa, wi, p))
                acc += p.a.re * p.a.re + p.a.im * p.a.im;
        }
        gain[c] += (float)acc;
    }
}

}  // namespace

hipError_t launch_coverage_diffraction(const DevScene& sc, const MatTable& mats, double lambda, const double* tx,
                                      const Antenna& txa, const Antenna& rxa, double gx0, double gy0, double gcell,
                                      double gz, int32_t gnx, int32_t gny, float* gain, hipStream_t s) {
    const int64_t cells = (int64_t)gnx * gny;
    if (cells <= 0 || sc.num_wedges <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((cells + kBlock - 1) / kBlock, 16384);
    hipLaunchKernelGGL(coverage_diffraction_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, sc, mats, lambda,
                       d3{tx[0], tx[1], tx[2]}, txa, rxa, gx0, gy0, gcell, gz, gnx, cells, gain);
    return hipGetLastError();
}

hipError_t launch_diffraction_paths(const PathArgs& a, const MatTable& mats, hipStream_t s) {
    const int64_t total = (int64_t)a.nrx * a.sc.num_wedges;
    if (total <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((total + kBlock - 1) / kBlock, 8192);
    hipLaunchKernelGGL(diffraction_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, a, mats);
    return hipGetLastError();
}

}  // namespace rt
