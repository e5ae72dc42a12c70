// Device-side math for the gfx950 kernels: small vector and complex types,
// antenna field patterns, Fresnel coefficients and the polarised field update
// at a specular reflection.
//
// Physics (paper Sec. II: materials are (eps_r, sigma) with mu_r = 1 and the
// polarised field components are transformed at every interaction; the
// formulas are the textbook ones):
//   eta     = eps_r - j sigma / (eps0 w)                (time dependence e^{+jwt})
//   s       = sqrt(eta - sin^2 theta_i), principal branch
//   r_perp  = (cos - s) / (cos + s),  r_par = (eta cos - s) / (eta cos + s)
//   d'      = d - 2 (d.n) n,  e_perp = d x n / |d x n|,
//   e_par_i = e_perp x d,  e_par_r = e_perp x d'
//   E'      = r_perp (E.e_perp) e_perp + r_par (E.e_par_i) e_par_r
// Antennas (Sec. II: yaw/pitch/roll orientation, preconfigured patterns):
//   R = Rz(yaw) Ry(pitch) Rx(roll); local direction R^T d -> (theta, phi);
//   field F = R (C_theta theta_hat + C_phi phi_hat); vertical polarisation
//   (C_phi = 0); isotropic C_theta = 1; TR 38.901 Table 7.3-1 element:
//   A = -min(-(A_V + A_H), 30), A_V = -min(12((theta-90)/65)^2, 30),
//   A_H = -min(12(phi/65)^2, 30) (degrees), C_theta = 10^((8 + A)/20).
#pragma once
#include <hip/hip_runtime.h>

#include "layout.h"

namespace rt {

constexpr double kPi = 3.14159265358979323846;
constexpr int kPatIso = 0;
constexpr int kPatTR38901 = 1;
constexpr int kPatDipole = 2;
constexpr int kMaxMaterials = 32;

struct MatTable {
    Mat m[kMaxMaterials];
};

// Antenna: orientation matrix (row-major) and pattern, in float and double.
struct Antenna {
    float R[9];
    int32_t pattern;
    int32_t pol;       // polarisation code: 0 V, 1 H, 2 +45 degrees, 3 -45 degrees
    double Rd[9];
};

// ---------------------------------------------------------------- float vec / complex
struct f3 {
    float x, y, z;
};
__device__ __forceinline__ f3 mk(float x, float y, float z) { return f3{x, y, z}; }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
    return f3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ f3 scale(f3 a, float s) { return f3{a.x * s, a.y * s, a.z * s}; }

struct cf {
    float re, im;
};
__device__ __forceinline__ cf cadd(cf a, cf b) { return cf{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return cf{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cf cmul(cf a, cf b) { return cf{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cf cmulr(cf a, float s) { return cf{a.re * s, a.im * s}; }
// fp32 field arithmetic uses the hardware reciprocal (about 1 ulp): the field
// feeds coverage sums compared at 1e-4 relative.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ cf cdiv(cf a, cf b) {
    const float inv = frcp(b.re * b.re + b.im * b.im);
    return cf{(a.re * b.re + a.im * b.im) * inv, (a.im * b.re - a.re * b.im) * inv};
}
__device__ __forceinline__ cf csqrt(cf z) {  // principal branch, cancellation-free
    const float r = sqrtf(z.re * z.re + z.im * z.im);
    if (z.re >= 0.0f) {
        const float re = sqrtf(0.5f * (r + z.re));
        return cf{re, re > 0.0f ? 0.5f * z.im * frcp(re) : 0.0f};
    }
    const float im = sqrtf(0.5f * (r - z.re));
    return cf{0.5f * fabsf(z.im) * frcp(im), copysignf(im, z.im)};
}

// ---------------------------------------------------------------- double vec / complex
struct d3 {
    double x, y, z;
};
__device__ __forceinline__ double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 cross(d3 a, d3 b) {
    return d3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ d3 sub(d3 a, d3 b) { return d3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ d3 add(d3 a, d3 b) { return d3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ d3 scale(d3 a, double s) { return d3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double norm(d3 a) { return sqrt(dot(a, a)); }

struct cd {
    double re, im;
};
__device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cmul(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cmulr(cd a, double s) { return cd{a.re * s, a.im * s}; }
__device__ __forceinline__ cd cdiv(cd a, cd b) {
    double den = b.re * b.re + b.im * b.im;
    return cd{(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}
__device__ __forceinline__ cd csqrt(cd z) {
    double r = hypot(z.re, z.im);
    if (z.re >= 0.0) {
        double re = sqrt(0.5 * (r + z.re));
        return cd{re, re > 0.0 ? z.im / (2.0 * re) : 0.0};
    }
    double im = sqrt(0.5 * (r - z.re));
    return cd{fabs(z.im) / (2.0 * im), copysign(im, z.im)};
}

// ---------------------------------------------------------------- antennas
// (cos zeta, sin zeta) of a polarisation code, exact in the given precision.
template <typename T>
__device__ __forceinline__ void pol_angle(int pol, T& c, T& s) {
    const T h = (T)0.70710678118654752440;
    switch (pol) {
        case 1: c = (T)0; s = (T)1; break;
        case 2: c = h; s = h; break;
        case 3: c = h; s = -h; break;
        default: c = (T)1; s = (T)0; break;
    }
}

__device__ __forceinline__ float tr38901_amp(float cos_t, float lx, float ly) {
    constexpr float kDeg = 57.29577951308232f;
    float th = acosf(fminf(fmaxf(cos_t, -1.0f), 1.0f)) * kDeg;
    float ph = atan2f(ly, lx) * kDeg;
    float av = -fminf(12.0f * ((th - 90.0f) / 65.0f) * ((th - 90.0f) / 65.0f), 30.0f);
    float ah = -fminf(12.0f * (ph / 65.0f) * (ph / 65.0f), 30.0f);
    float a = -fminf(-(av + ah), 30.0f);
    return exp10f((8.0f + a) * 0.05f);
}

// Field vector of antenna `ant` towards global unit direction d.
__device__ __forceinline__ f3 antenna_field(const Antenna& ant, f3 d) {
    const float* R = ant.R;
    float lx = R[0] * d.x + R[3] * d.y + R[6] * d.z;
    float ly = R[1] * d.x + R[4] * d.y + R[7] * d.z;
    float lz = R[2] * d.x + R[5] * d.y + R[8] * d.z;
    const float rho2 = lx * lx + ly * ly;
    float cph = 1.0f, sph = 0.0f, rho = 0.0f;
    if (rho2 > 0.0f) {
        const float ir = __builtin_amdgcn_rsqf(rho2);
        rho = rho2 * ir;
        cph = lx * ir;
        sph = ly * ir;
    }
    float g = 1.0f;
    if (ant.pattern == kPatTR38901) g = tr38901_amp(lz, lx, ly);
    else if (ant.pattern == kPatDipole) g = 1.22474487f * rho;  // sqrt(1.5) sin(theta)
    float zc, zs;
    pol_angle(ant.pol, zc, zs);
    const float ct = g * zc, cp = g * zs;  // theta-hat and phi-hat components
    float tx = ct * lz * cph - cp * sph, ty = ct * lz * sph + cp * cph, tz = -ct * rho;
    return f3{R[0] * tx + R[1] * ty + R[2] * tz, R[3] * tx + R[4] * ty + R[5] * tz, R[6] * tx + R[7] * ty + R[8] * tz};
}

__device__ __forceinline__ double tr38901_amp_d(double cos_t, double lx, double ly) {
    constexpr double kDeg = 180.0 / kPi;
    double th = acos(fmin(fmax(cos_t, -1.0), 1.0)) * kDeg;
    double ph = atan2(ly, lx) * kDeg;
    double av = -fmin(12.0 * ((th - 90.0) / 65.0) * ((th - 90.0) / 65.0), 30.0);
    double ah = -fmin(12.0 * (ph / 65.0) * (ph / 65.0), 30.0);
    double a = -fmin(-(av + ah), 30.0);
    return exp10((8.0 + a) / 20.0);
}

__device__ __forceinline__ d3 antenna_field(const Antenna& ant, d3 d) {
    const double* R = ant.Rd;
    double lx = R[0] * d.x + R[3] * d.y + R[6] * d.z;
    double ly = R[1] * d.x + R[4] * d.y + R[7] * d.z;
    double lz = R[2] * d.x + R[5] * d.y + R[8] * d.z;
    double rho = sqrt(lx * lx + ly * ly);
    double cph = 1.0, sph = 0.0;
    if (rho > 0.0) {
        cph = lx / rho;
        sph = ly / rho;
    }
    double g = 1.0;
    if (ant.pattern == kPatTR38901) g = tr38901_amp_d(lz, lx, ly);
    else if (ant.pattern == kPatDipole) g = 1.2247448713915890 * rho;  // sqrt(1.5) sin(theta)
    double zc, zs;
    pol_angle(ant.pol, zc, zs);
    const double ct = g * zc, cp = g * zs;
    double tx = ct * lz * cph - cp * sph, ty = ct * lz * sph + cp * cph, tz = -ct * rho;
    return d3{R[0] * tx + R[1] * ty + R[2] * tz, R[3] * tx + R[4] * ty + R[5] * tz, R[6] * tx + R[7] * ty + R[8] * tz};
}

// Draw c of the SplitMix64 stream seeded with s (the generator's stateless
// form: the state after c + 1 steps is s + (c + 1) g), and a uniform in [0, 1)
// from its top 53 bits.
__device__ __forceinline__ uint64_t splitmix64(uint64_t s, uint64_t c) {
    uint64_t z = s + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double uniform01(uint64_t s, uint64_t c) {
    return (double)(splitmix64(s, c) >> 11) * 0x1p-53;
}

// Cosine-weighted (Lambertian) direction around the unit normal n from two
// uniforms: frame t = normalize(n x a) with a the coordinate axis least aligned
// with n (lowest index on ties), b = n x t; direction
// sqrt(u1) (cos 2 pi u2 t + sin 2 pi u2 b) + sqrt(1 - u1) n.
__device__ __forceinline__ d3 lambert_dir(d3 n, double u1, double u2) {
    const double ax = fabs(n.x), ay = fabs(n.y), az = fabs(n.z);
    const d3 a = (ax <= ay && ax <= az) ? d3{1.0, 0.0, 0.0} : (ay <= az ? d3{0.0, 1.0, 0.0} : d3{0.0, 0.0, 1.0});
    d3 t = cross(n, a);
    t = scale(t, 1.0 / norm(t));
    const d3 b = cross(n, t);
    const double r = sqrt(u1), z = sqrt(1.0 - u1);
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    return add(add(scale(t, r * c), scale(b, r * s)), scale(n, z));
}

// Direction of Fibonacci-lattice ray i of N (Sec. II-B): z = 1 - (2i+1)/N,
// azimuth 2 pi frac(i g) with frac(i g) = (i * 0x9E3779B97F4A7C15 mod 2^64) / 2^64.
__device__ __forceinline__ d3 fib_dir(int64_t i, int64_t N) {
    const double z = 1.0 - (2.0 * (double)i + 1.0) / (double)N;
    const double rho = sqrt((1.0 - z) * (1.0 + z));
    const uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull;
    double s, c;
    sincospi(2.0 * ((double)h * 0x1p-64), &s, &c);  // angle 2 pi frac(i g)
    return d3{rho * c, rho * s, z};
}

// ---------------------------------------------------------------- Fresnel
__device__ __forceinline__ void fresnel(const Mat& m, float cos_i, cf& r_perp, cf& r_par) {
    if (m.pec) {
        r_perp = cf{-1.0f, 0.0f};
        r_par = cf{1.0f, 0.0f};
        return;
    }
    cf eta{m.eta_re, m.eta_im};
    float sin2 = 1.0f - cos_i * cos_i;
    cf s = csqrt(cf{eta.re - sin2, eta.im});
    cf c{cos_i, 0.0f};
    r_perp = cdiv(csub(c, s), cadd(c, s));
    cf ec = cmulr(eta, cos_i);
    r_par = cdiv(csub(ec, s), cadd(ec, s));
}

__device__ __forceinline__ void fresnel(const Mat& m, double cos_i, cd& r_perp, cd& r_par) {
    if (m.pec) {
        r_perp = cd{-1.0, 0.0};
        r_par = cd{1.0, 0.0};
        return;
    }
    cd eta{m.eta_re_d, m.eta_im_d};
    double sin2 = 1.0 - cos_i * cos_i;
    cd s = csqrt(cd{eta.re - sin2, eta.im});
    cd c{cos_i, 0.0};
    r_perp = cdiv(csub(c, s), cadd(c, s));
    cd ec = cmulr(eta, cos_i);
    r_par = cdiv(csub(ec, s), cadd(ec, s));
}

// Field factor of a specular reflection on a scattering material: the
// reflected power splits into S^2 diffuse and 1 - S^2 specular (the Lambertian
// model of the coverage maps), so a specular path carries sqrt(1 - S^2) per
// reflection (1 when the material does not scatter).
__device__ __forceinline__ double specular_share(const Mat& m) {
    const double S = (double)m.scat;
    return sqrt(1.0 - S * S);
}

// Unit vector perpendicular to the plane of incidence; any unit vector
// orthogonal to d at normal incidence (the result does not depend on it).
__device__ __forceinline__ d3 perp_basis(d3 d, d3 n) {
    d3 e = cross(d, n);
    double l = norm(e);
    if (l < 1e-12) {
        double ax = fabs(d.x), ay = fabs(d.y), az = fabs(d.z);
        d3 a = (ax <= ay && ax <= az) ? d3{1, 0, 0} : ((ay <= az) ? d3{0, 1, 0} : d3{0, 0, 1});
        e = sub(a, scale(d, dot(a, d)));
        l = norm(e);
    }
    return scale(e, 1.0 / l);
}

}  // namespace rt
