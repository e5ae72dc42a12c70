// Gradient of received power for gfx950 (paper Sec. I and II: channel
// responses are differentiable with respect to material properties,
// antenna orientations and positions; Sec. III-A learns (eps_r, sigma) and
// Sec. III-B optimises the transmitter orientation by gradient steps).
//
// Input: the paths of one transmitter as face sequences (the checkpoint kept
// by the forward pass).  One thread per (rx, path) recomputes the path in
// fp64 and differentiates its power |a|^2:
//   * transmitter position (x, y, z) and orientation (yaw, pitch) with
//     forward-mode dual numbers carrying 5 tangents through the images,
//     reflection points, directions, length, Fresnel coefficients, field
//     bases and the transmit pattern;
//   * material (eps_r, sigma) of every face on the path by one reverse sweep:
//     a = g_K^T R_K ... R_1 E_0 is linear in each r_perp/r_par, so
//     da/dr_perp_k = (g_k . e_perp) (e_perp . E_{k-1}),
//     da/dr_par_k  = (g_k . e_par_r) (e_par_i . E_{k-1}), with
//     g_{k-1} = R_k^T g_k, dr_perp/deta = -cos / (s (cos + s)^2),
//     dr_par/deta = cos (eta - 2 sin^2) / (s (eta cos + s)^2),
//     deta/deps_r = 1, deta/dsigma = -j / (eps0 w).
// Power derivatives dP/dtheta = 2 Re(conj(a) da/dtheta) are contracted with
// the upstream adjoint dL/dP_r and accumulated with fp64 atomics.
#include "traverse.h"

namespace rt {
namespace {

constexpr int NT = 5;
constexpr int kMaxK = 8;
constexpr double kEps0 = 8.8541878128e-12;

struct D {
    double v;
    double d[NT];
};
__device__ __forceinline__ D dc(double v) {
    D r;
    r.v = v;
    for (int i = 0; i < NT; ++i) r.d[i] = 0.0;
    return r;
}
__device__ __forceinline__ D operator+(D a, D b) {
    D r;
    r.v = a.v + b.v;
    for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
__device__ __forceinline__ D operator-(D a, D b) {
    D r;
    r.v = a.v - b.v;
    for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
__device__ __forceinline__ D operator-(D a) {
    D r;
    r.v = -a.v;
    for (int i = 0; i < NT; ++i) r.d[i] = -a.d[i];
    return r;
}
__device__ __forceinline__ D operator*(D a, D b) {
    D r;
    r.v = a.v * b.v;
    for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
__device__ __forceinline__ D operator*(D a, double s) {
    D r;
    r.v = a.v * s;
    for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] * s;
    return r;
}
__device__ __forceinline__ D operator/(D a, D b) {
    D r;
    r.v = a.v / b.v;
    const double ib = 1.0 / b.v;
    for (int i = 0; i < NT; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
    return r;
}
__device__ __forceinline__ D dsqrt(D a) {
    D r;
    r.v = sqrt(a.v);
    const double k = r.v > 0.0 ? 0.5 / r.v : 0.0;
    for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] * k;
    return r;
}
__device__ __forceinline__ D dfun(D a, double v, double dv) {
    D r;
    r.v = v;
    for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] * dv;
    return r;
}
__device__ __forceinline__ D dcos(D a) { return dfun(a, cos(a.v), -sin(a.v)); }
__device__ __forceinline__ D dsin(D a) { return dfun(a, sin(a.v), cos(a.v)); }
__device__ __forceinline__ D dacos(D a) {
    const double x = fmin(fmax(a.v, -1.0), 1.0);
    const double den = sqrt(fmax(1.0 - x * x, 1e-300));
    return dfun(a, acos(x), -1.0 / den);
}
__device__ __forceinline__ D datan2(D y, D x) {
    D r;
    r.v = atan2(y.v, x.v);
    const double den = x.v * x.v + y.v * y.v;
    for (int i = 0; i < NT; ++i) r.d[i] = den > 0.0 ? (x.v * y.d[i] - y.v * x.d[i]) / den : 0.0;
    return r;
}
__device__ __forceinline__ D dexp10(D a) {
    const double v = exp10(a.v);
    return dfun(a, v, v * 2.302585092994045684);
}
__device__ __forceinline__ D dmin(D a, D b) { return a.v <= b.v ? a : b; }

struct D3 {
    D x, y, z;
};
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return D3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return D3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 operator*(D3 a, D s) { return D3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ D3 operator*(D3 a, double s) { return D3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ D ddot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D ddot(D3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 dcross(D3 a, D3 b) {
    return D3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ D3 dcross(D3 a, d3 b) {
    return D3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ D3 dconst(d3 a) { return D3{dc(a.x), dc(a.y), dc(a.z)}; }
__device__ __forceinline__ d3 val(D3 a) { return d3{a.x.v, a.y.v, a.z.v}; }
__device__ __forceinline__ D dnorm(D3 a) { return dsqrt(ddot(a, a)); }

// complex dual
struct C {
    D re, im;
};
__device__ __forceinline__ C operator+(C a, C b) { return C{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ C operator-(C a, C b) { return C{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ C operator*(C a, C b) { return C{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ C operator*(C a, D s) { return C{a.re * s, a.im * s}; }
__device__ __forceinline__ C operator/(C a, C b) {
    D den = b.re * b.re + b.im * b.im;
    return C{(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}
__device__ __forceinline__ C csqrt_d(C z) {
    D r = dsqrt(z.re * z.re + z.im * z.im);
    if (z.re.v >= 0.0) {
        D re = dsqrt((r + z.re) * 0.5);
        return C{re, z.im / (re * 2.0)};
    }
    D im = dsqrt((r - z.re) * 0.5);
    D absim = z.im.v >= 0.0 ? z.im : -z.im;
    return C{absim / (im * 2.0), z.im.v >= 0.0 ? im : -im};
}
struct C3 {
    C x, y, z;
};
__device__ __forceinline__ C cdot(C3 a, D3 b) { return C{ddot(D3{a.x.re, a.y.re, a.z.re}, b), ddot(D3{a.x.im, a.y.im, a.z.im}, b)}; }
__device__ __forceinline__ C3 cscale(D3 v, C s) {
    return C3{C{v.x * s.re, v.x * s.im}, C{v.y * s.re, v.y * s.im}, C{v.z * s.re, v.z * s.im}};
}
__device__ __forceinline__ C3 cadd3(C3 a, C3 b) { return C3{a.x + b.x, a.y + b.y, a.z + b.z}; }

struct DRot {
    D R[9];
};
__device__ DRot drot(D yaw, D pitch, D roll) {
    D cy = dcos(yaw), sy = dsin(yaw), cp = dcos(pitch), sp = dsin(pitch), cr = dcos(roll), sr = dsin(roll);
    DRot o;
    o.R[0] = cy * cp; o.R[1] = cy * sp * sr - sy * cr; o.R[2] = cy * sp * cr + sy * sr;
    o.R[3] = sy * cp; o.R[4] = sy * sp * sr + cy * cr; o.R[5] = sy * sp * cr - cy * sr;
    o.R[6] = -sp;     o.R[7] = cp * sr;                o.R[8] = cp * cr;
    return o;
}

__device__ D3 dantenna(const DRot& Rr, int pattern, D3 d, int pol = 0) {
    const D* R = Rr.R;
    D lx = R[0] * d.x + R[3] * d.y + R[6] * d.z;
    D ly = R[1] * d.x + R[4] * d.y + R[7] * d.z;
    D lz = R[2] * d.x + R[5] * d.y + R[8] * d.z;
    D rho = dsqrt(lx * lx + ly * ly);
    D cph = dc(1.0), sph = dc(0.0);
    if (rho.v > 0.0) {
        cph = lx / rho;
        sph = ly / rho;
    }
    D c = dc(1.0);
    if (pattern == kPatTR38901) {
        const double kDeg = 180.0 / kPi;
        D th = dacos(lz) * kDeg;
        D ph = datan2(ly, lx) * kDeg;
        D u = (th - dc(90.0)) * (1.0 / 65.0);
        D w = ph * (1.0 / 65.0);
        D av = -dmin(u * u * 12.0, dc(30.0));
        D ah = -dmin(w * w * 12.0, dc(30.0));
        D a = -dmin(-(av + ah), dc(30.0));
        c = dexp10((a + dc(8.0)) * (1.0 / 20.0));
    } else if (pattern == kPatDipole) {
        c = rho * 1.2247448713915890;  // sqrt(1.5) sin(theta)
    }
    double zc, zs;
    pol_angle(pol, zc, zs);
    const D ct = c * zc, cp = c * zs;
    D tx = ct * lz * cph - cp * sph, ty = ct * lz * sph + cp * cph, tz = -(ct * rho);
    return D3{R[0] * tx + R[1] * ty + R[2] * tz, R[3] * tx + R[4] * ty + R[5] * tz, R[6] * tx + R[7] * ty + R[8] * tz};
}

__device__ D3 dperp(D3 d, d3 n) {
    D3 e = dcross(d, n);
    D l = dnorm(e);
    if (l.v < 1e-12) {  // normal incidence: any unit vector orthogonal to d (result independent of it)
        d3 dv = val(d);
        double ax = fabs(dv.x), ay = fabs(dv.y), az = fabs(dv.z);
        d3 a = (ax <= ay && ax <= az) ? d3{1, 0, 0} : ((ay <= az) ? d3{0, 1, 0} : d3{0, 0, 1});
        e = dconst(a) - d * ddot(d, a);
        l = dnorm(e);
    }
    return e * (dc(1.0) / l);
}

__device__ __forceinline__ cd cdotv(const cd* g, d3 v) {
    return cd{g[0].re * v.x + g[1].re * v.y + g[2].re * v.z, g[0].im * v.x + g[1].im * v.y + g[2].im * v.z};
}

__global__ void power_grad_kernel(GradArgs g, MatTable mats) {
    const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= (int64_t)g.nrx * g.P) return;
    const int r = (int)(item / g.P);
    const int K = g.depth[item];
    if (K < 0 || K > g.fd || K > kMaxK) return;  // empty slot (or not a path of this depth range)
    // adjoint of the path coefficient: the contribution of the path is
    // Re(gc * da/dtheta), gc given (coef_adj) or 2 w conj(a) for the power
    // |a|^2 weighted by the upstream w = dL/dP_r
    const double w_up = g.coef_adj ? 0.0 : g.dL_dP[r];
    if (g.coef_adj ? (g.coef_adj[2 * item] == 0.0 && g.coef_adj[2 * item + 1] == 0.0) : w_up == 0.0) return;
    int fc[kMaxK];
    for (int i = 0; i < K; ++i) {
        fc[i] = g.faces[item * g.fd + i];
        if (fc[i] < 0 || fc[i] >= g.sc.num_faces) return;
    }
    // seeds: tangents 0..2 tx position, 3 yaw, 4 pitch
    D3 tx{dc(g.tx[0]), dc(g.tx[1]), dc(g.tx[2])};
    tx.x.d[0] = 1.0;
    tx.y.d[1] = 1.0;
    tx.z.d[2] = 1.0;
    D yaw = dc(g.yaw), pitch = dc(g.pitch);
    yaw.d[3] = 1.0;
    pitch.d[4] = 1.0;
    const DRot Rt = drot(yaw, pitch, dc(g.roll));
    const d3 rx{g.rx[3 * r], g.rx[3 * r + 1], g.rx[3 * r + 2]};
    D3 I[kMaxK + 1];
    I[0] = tx;
    for (int k = 1; k <= K; ++k) {
        const Face F = g.sc.faces[fc[k - 1]];
        const d3 n{F.n[0], F.n[1], F.n[2]}, q{F.q[0], F.q[1], F.q[2]};
        I[k] = I[k - 1] - dconst(n) * (ddot(I[k - 1] - dconst(q), n) * 2.0);
    }
    D3 X[kMaxK + 2];
    X[0] = tx;
    X[K + 1] = dconst(rx);
    for (int k = K; k >= 1; --k) {
        const Face F = g.sc.faces[fc[k - 1]];
        const d3 n{F.n[0], F.n[1], F.n[2]}, q{F.q[0], F.q[1], F.q[2]};
        const D3 A = X[k + 1];
        const D t = ddot(dconst(q) - A, n) / ddot(I[k] - A, n);
        X[k] = A + (I[k] - A) * t;
    }
    D3 dir[kMaxK + 1];
    D L = dc(0.0);
    for (int k = 0; k <= K; ++k) {
        const D3 s = X[k + 1] - X[k];
        const D l = dnorm(s);
        L = L + l;
        dir[k] = s * (dc(1.0) / l);
    }
    const D3 F0 = dantenna(Rt, g.tx_pattern, dir[0], g.tx_pol);
    C3 E{C{F0.x, dc(0.0)}, C{F0.y, dc(0.0)}, C{F0.z, dc(0.0)}};
    // values kept for the material sweep
    d3 ep_v[kMaxK], eli_v[kMaxK], elr_v[kMaxK];
    cd aperp[kMaxK], apar[kMaxK], rp_v[kMaxK], rl_v[kMaxK], drp[kMaxK], drl[kMaxK];
    int mat_k[kMaxK];
    for (int k = 1; k <= K; ++k) {
        const Face F = g.sc.faces[fc[k - 1]];
        d3 n{F.n[0], F.n[1], F.n[2]};
        const D3 din = dir[k - 1], dout = dir[k];
        if (ddot(din, n).v > 0.0) n = scale(n, -1.0);
        const D cos_i = -ddot(din, n);
        const Mat m = mats.m[F.mat];
        C rp, rl;
        cd drp_v{0, 0}, drl_v{0, 0};
        if (m.pec) {
            rp = C{dc(-1.0), dc(0.0)};
            rl = C{dc(1.0), dc(0.0)};
        } else {
            const C eta{dc(m.eta_re_d), dc(m.eta_im_d)};
            const D sin2 = dc(1.0) - cos_i * cos_i;
            const C s = csqrt_d(C{eta.re - sin2, eta.im});
            const C c{cos_i, dc(0.0)};
            rp = (c - s) / (c + s);
            const C ec = eta * cos_i;
            rl = (ec - s) / (ec + s);
            // d r / d eta (values)
            const cd sv{s.re.v, s.im.v}, cv{cos_i.v, 0.0}, ev{m.eta_re_d, m.eta_im_d};
            const cd cps = cadd(cv, sv), ecs = cadd(cmulr(ev, cos_i.v), sv);
            drp_v = cdiv(cd{-cos_i.v, 0.0}, cmul(sv, cmul(cps, cps)));
            const cd num = cmulr(csub(ev, cd{2.0 * sin2.v, 0.0}), cos_i.v);
            drl_v = cdiv(num, cmul(sv, cmul(ecs, ecs)));
        }
        {  // specular share of a scattering material (a constant factor)
            const double share = specular_share(m);
            rp = rp * dc(share);
            rl = rl * dc(share);
            drp_v = cmulr(drp_v, share);
            drl_v = cmulr(drl_v, share);
        }
        const D3 ep = dperp(din, n);
        const D3 eli = dcross(ep, din), elr = dcross(ep, dout);
        const C ap = cdot(E, ep), al = cdot(E, eli);
        ep_v[k - 1] = val(ep);
        eli_v[k - 1] = val(eli);
        elr_v[k - 1] = val(elr);
        aperp[k - 1] = cd{ap.re.v, ap.im.v};
        apar[k - 1] = cd{al.re.v, al.im.v};
        rp_v[k - 1] = cd{rp.re.v, rp.im.v};
        rl_v[k - 1] = cd{rl.re.v, rl.im.v};
        drp[k - 1] = drp_v;
        drl[k - 1] = drl_v;
        mat_k[k - 1] = F.mat;
        E = cadd3(cscale(ep, rp * ap), cscale(elr, rl * al));
    }
    const D3 mdK = dir[K] * -1.0;
    // receive pattern: receiver pose is not a differentiated parameter
    const Antenna ra = g.rx_ant[r];
    DRot Rr;
    for (int i = 0; i < 9; ++i) Rr.R[i] = dc(ra.Rd[i]);
    const D3 Fr = dantenna(Rr, ra.pattern, mdK, ra.pol);
    const D amp = dc(g.lambda / (4.0 * kPi)) / L;
    const C pr = cdot(E, Fr);
    const C a{pr.re * amp, pr.im * amp};
    const double gre = g.coef_adj ? g.coef_adj[2 * item] : 2.0 * w_up * a.re.v;
    const double gim = g.coef_adj ? g.coef_adj[2 * item + 1] : -2.0 * w_up * a.im.v;
    double* out = g.grad;
    const int base = 2 * g.nm;
    for (int i = 0; i < NT; ++i) atomicAdd(out + base + i, gre * a.re.d[i] - gim * a.im.d[i]);
    // material sweep
    cd gv[3] = {cd{amp.v * Fr.x.v, 0.0}, cd{amp.v * Fr.y.v, 0.0}, cd{amp.v * Fr.z.v, 0.0}};
    const double w = 2.0 * kPi * g.freq;
    for (int k = K; k >= 1; --k) {
        const int i = k - 1;
        const cd gp = cdotv(gv, ep_v[i]);
        const cd gl = cdotv(gv, elr_v[i]);
        const cd da = cadd(cmul(cmul(gp, aperp[i]), drp[i]), cmul(cmul(gl, apar[i]), drl[i]));
        // d/deps_r: Re(gc da); d/dsigma: Re(gc da (-j / (eps0 w))) = Im(gc da) / (eps0 w)
        const double re_gd = gre * da.re - gim * da.im;
        const double im_gd = gre * da.im + gim * da.re;
        const double dsig = 1.0 / (kEps0 * w);
        if (drp[i].re != 0.0 || drp[i].im != 0.0 || drl[i].re != 0.0 || drl[i].im != 0.0) {
            atomicAdd(out + 2 * mat_k[i], re_gd);
            atomicAdd(out + 2 * mat_k[i] + 1, im_gd * dsig);
        }
        // g <- R_k^T g
        const cd p1 = cmul(rp_v[i], gp), p2 = cmul(rl_v[i], gl);
        const d3 e1 = ep_v[i], e2 = eli_v[i];
        gv[0] = cadd(cmulr(p1, e1.x), cmulr(p2, e2.x));
        gv[1] = cadd(cmulr(p1, e1.y), cmulr(p2, e2.y));
        gv[2] = cadd(cmulr(p1, e1.z), cmulr(p2, e2.z));
    }
}

// ------------------------------------------------------------------ coverage
// Gradient of the path gain summed over a region of coverage-map cells with
// respect to the radio materials and the transmitter orientation (the
// coverage analogue of the received-power gradient; Sec. III-B optimises a
// transmitter orientation by gradient steps).  Ray geometry does not depend
// on these parameters, so the recorded hits (triangle and distance per
// segment) fix every ray; one thread per ray replays it in fp64 with the
// same formulas as the shoot-and-bounce kernel and carries, beside the field
// E, its tangents dE/dtheta:
//   * at launch, d F_tx / d(yaw, pitch) from the dual-number transmit pattern;
//   * at a reflection off material m, E' = R E gives
//     dE'/dtheta = R dE/dtheta + [theta of m] (dR/d eta) E (d eta/d theta),
//     with dR/d eta from d r_perp / d eta and d r_par / d eta as above;
//   * every crossing of the grid plane inside the region adds
//     w = wscale |F_rx . E|^2 / |d_z| and dw = wscale 2 Re(conj(a) F_rx . dE) / |d_z|.
__device__ __forceinline__ cd dot3(const cd* v, d3 u) {
    return cd{v[0].re * u.x + v[1].re * u.y + v[2].re * u.z, v[0].im * u.x + v[1].im * u.y + v[2].im * u.z};
}

__global__ __launch_bounds__(256) void coverage_grad_kernel(CovGradArgs g, MatTable mats) {
    __shared__ double red[4][1 + kCovT];
    double acc[1 + kCovT];
#pragma unroll
    for (int i = 0; i <= kCovT; ++i) acc[i] = 0.0;
    const int yaw_t = 2 * kCovMaxMat, pitch_t = 2 * kCovMaxMat + 1;
    // transmit pattern tangents are those of dantenna's slots 3 (yaw) and 4 (pitch)
    D yaw = dc(g.yaw), pitch = dc(g.pitch);
    yaw.d[3] = 1.0;
    pitch.d[4] = 1.0;
    const DRot Rt = drot(yaw, pitch, dc(g.roll));
    const double dsig = 1.0 / (kEps0 * g.omega);
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < g.count;
         j += (int64_t)gridDim.x * blockDim.x) {
        d3 d = fib_dir(g.begin + j * g.stride, g.num_rays);
        d3 o{g.tx[0], g.tx[1], g.tx[2]};
        const D3 F0 = dantenna(Rt, g.tx_pattern, dconst(d), g.tx_pol);
        cd E[3] = {cd{F0.x.v, 0.0}, cd{F0.y.v, 0.0}, cd{F0.z.v, 0.0}};
        cd dE[kCovT][3];
#pragma unroll
        for (int i = 0; i < kCovT; ++i) dE[i][0] = dE[i][1] = dE[i][2] = cd{0.0, 0.0};
        dE[yaw_t][0] = cd{F0.x.d[3], 0.0};
        dE[yaw_t][1] = cd{F0.y.d[3], 0.0};
        dE[yaw_t][2] = cd{F0.z.d[3], 0.0};
        dE[pitch_t][0] = cd{F0.x.d[4], 0.0};
        dE[pitch_t][1] = cd{F0.y.d[4], 0.0};
        dE[pitch_t][2] = cd{F0.z.d[4], 0.0};
        for (int k = 0; k <= g.max_depth; ++k) {
            const int32_t tri = g.hit_tri[(int64_t)k * g.count + j];
            if (tri == -2) break;
            const double t = g.hit_t[(int64_t)k * g.count + j];
            const double dz = d.z;
            if (fabs(dz) >= 1e-12) {
                const double tc = (g.gz - o.z) / dz;
                if (tc > 0.0 && tc < t) {
                    const double x = o.x + tc * d.x, y = o.y + tc * d.y;
                    const double fx = floor((x - g.gx0) / g.gcell), fy = floor((y - g.gy0) / g.gcell);
                    if (fx >= 0.0 && fx < (double)g.gnx && fy >= 0.0 && fy < (double)g.gny) {
                        const int64_t cell = (int64_t)fy * g.gnx + (int64_t)fx;
                        if (!g.region || g.region[cell]) {
                            const d3 fr = antenna_field(g.rx_ant, d3{-d.x, -d.y, -d.z});
                            const cd a = dot3(E, fr);
                            const double w0 = g.wscale / fabs(dz);
                            acc[0] += w0 * (a.re * a.re + a.im * a.im);
#pragma unroll
                            for (int i = 0; i < kCovT; ++i) {
                                const cd da = dot3(dE[i], fr);
                                acc[1 + i] += 2.0 * w0 * (a.re * da.re + a.im * da.im);
                            }
                        }
                    }
                }
            }
            if (tri < 0 || k == g.max_depth || tri >= g.sc.nt) break;
            const Shade sh = g.sc.shades[g.sc.leaf_of_input[tri]];
            d3 n{sh.n[0], sh.n[1], sh.n[2]};
            if (dot(d, n) > 0.0) n = scale(n, -1.0);
            const double cos_i = -dot(d, n);
            const d3 dr = add(d, scale(n, 2.0 * cos_i));
            const d3 p = add(o, scale(d, t));
            const d3 ep = perp_basis(d, n);
            const d3 eli = cross(ep, d);
            // the outgoing direction and transverse basis: specular, or diffuse
            // with the forward kernel's draws (they depend on no parameter)
            d3 dout = dr, epo = ep, elr = cross(ep, dr);
            if (mats.m[sh.mat].scat > 0.0f) {
                const uint64_t ri = (uint64_t)(g.begin + j * g.stride);
                const uint64_t c0 = (ri * (uint64_t)(g.max_depth + 1) + (uint64_t)k) * 3ull;
                const double S = (double)mats.m[sh.mat].scat;
                if (uniform01(g.scat_seed, c0) < S * S) {
                    dout = lambert_dir(n, uniform01(g.scat_seed, c0 + 1), uniform01(g.scat_seed, c0 + 2));
                    epo = perp_basis(dout, n);
                    elr = cross(epo, dout);
                }
            }
            const Mat mt = mats.m[sh.mat];
            cd rp, rl;
            fresnel(mt, cos_i, rp, rl);
            cd drp{0.0, 0.0}, drl{0.0, 0.0};
            if (!mt.pec) {
                const cd eta{mt.eta_re_d, mt.eta_im_d};
                const double sin2 = 1.0 - cos_i * cos_i;
                const cd s = csqrt(cd{eta.re - sin2, eta.im});
                const cd cps = cadd(cd{cos_i, 0.0}, s), ecs = cadd(cmulr(eta, cos_i), s);
                drp = cdiv(cd{-cos_i, 0.0}, cmul(s, cmul(cps, cps)));
                drl = cdiv(cmulr(csub(eta, cd{2.0 * sin2, 0.0}), cos_i), cmul(s, cmul(ecs, ecs)));
            }
            const cd ap = dot3(E, ep), al = dot3(E, eli);
            const cd sp = cmul(rp, ap), sl = cmul(rl, al);
            const cd dsp = cmul(drp, ap), dsl = cmul(drl, al);  // d(r a)/d eta
#pragma unroll
            for (int i = 0; i < kCovT; ++i) {
                const cd api = cmul(rp, dot3(dE[i], ep)), ali = cmul(rl, dot3(dE[i], eli));
                dE[i][0] = cadd(cmulr(api, epo.x), cmulr(ali, elr.x));
                dE[i][1] = cadd(cmulr(api, epo.y), cmulr(ali, elr.y));
                dE[i][2] = cadd(cmulr(api, epo.z), cmulr(ali, elr.z));
            }
            if (sh.mat < kCovMaxMat && !mt.pec) {
                const cd de[3] = {cadd(cmulr(dsp, epo.x), cmulr(dsl, elr.x)), cadd(cmulr(dsp, epo.y), cmulr(dsl, elr.y)),
                                  cadd(cmulr(dsp, epo.z), cmulr(dsl, elr.z))};
                const cd mj{0.0, -dsig};  // d eta / d sigma = -j / (eps0 w)
#pragma unroll
                for (int m = 0; m < kCovMaxMat; ++m)
                    if (m == sh.mat) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            dE[2 * m][c] = cadd(dE[2 * m][c], de[c]);
                            dE[2 * m + 1][c] = cadd(dE[2 * m + 1][c], cmul(de[c], mj));
                        }
                    }
            }
            E[0] = cadd(cmulr(sp, epo.x), cmulr(sl, elr.x));
            E[1] = cadd(cmulr(sp, epo.y), cmulr(sl, elr.y));
            E[2] = cadd(cmulr(sp, epo.z), cmulr(sl, elr.z));
            o = p;
            d = dout;
        }
    }
    // block reduction (wave shuffles, then the four waves through LDS), one
    // fp64 atomic per block and output
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i <= kCovT; ++i) {
        double v = acc[i];
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][i] = v;
    }
    __syncthreads();
    if (threadIdx.x <= kCovT) {
        // slot 0 the region sum, 1 + 2m + {0, 1} material m, then yaw, pitch;
        // out has 2 nm + 3 entries in the same order
        const int i = threadIdx.x;
        int o = -1;
        if (i == 0) o = 0;
        else if (i - 1 < 2 * g.nm) o = i;
        else if (i - 1 == yaw_t) o = 1 + 2 * g.nm;
        else if (i - 1 == pitch_t) o = 2 + 2 * g.nm;
        const double v = red[0][i] + red[1][i] + red[2][i] + red[3][i];
        if (o >= 0 && v != 0.0) atomicAdd(g.out + o, v);
    }
}

}  // namespace

hipError_t launch_power_grad(const GradArgs& a, const MatTable& mats, hipStream_t s) {
    const int64_t n = (int64_t)a.nrx * a.P;
    const int64_t blocks = (n + 127) / 128;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(power_grad_kernel, dim3((unsigned)blocks), dim3(128), 0, s, a, mats);
    return hipGetLastError();
}

hipError_t launch_coverage_grad(const CovGradArgs& a, const MatTable& mats, int grid, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    const int64_t need = (a.count + 255) / 256;
    const unsigned blocks = (unsigned)(need < grid ? need : grid);
    hipLaunchKernelGGL(coverage_grad_kernel, dim3(blocks), dim3(256), 0, s, a, mats);
    return hipGetLastError();
}

}  // namespace rt
