// Shoot-and-bounce kernels for gfx950 (paper Sec. II-B: rays shot in
// Fibonacci-lattice directions propagate through the scene with specular
// reflections until the maximum depth; Sec. II-A: coverage maps of path
// gain; Sec. II: per-interaction transformation of the polarised field).
//
// One launch per bounce ("wavefront" organisation):
//   bounce 0 generates rays in coherence order and traces them;
//   bounce k > 0 reads the compacted queue of rays that survived bounce k-1.
// Each launch runs a persistent, wave-strided loop.  Per ray: closest hit
// (fp32 conservative slab tests on a 4-wide BVH with a per-lane LDS stack,
// fp64 Moller-Trumbore on triangles), coverage deposit of the segment, then
// Fresnel reflection of the field and a wave-ballot compaction into the next
// queue (one atomic per wave).
#include "traverse.h"

namespace rt {
namespace {

// q = floor(x / F), r = x - q F for 0 <= x < 2^52 and F < 2^26, using the
// precomputed double 1/F and one correction step.
__device__ __forceinline__ void divmod(int64_t x, int64_t F, double invF, int64_t& q, int64_t& r) {
    q = (int64_t)((double)x * invF);
    r = x - q * F;
    if (r < 0) {
        q -= 1;
        r += F;
    } else if (r >= F) {
        q += 1;
        r -= F;
    }
}

// Traced position j -> lattice position.  With a band permutation, positions
// are taken in bands of F consecutive indices (a thin latitude ring); inside
// a band, rank r maps to offset r * G mod F (G the preceding Fibonacci
// number), which walks the ring in azimuth order, so 64 consecutive positions
// form a compact patch of directions.
__device__ __forceinline__ int64_t lattice_position(const SbrArgs& a, int64_t j) {
    if (a.perm_f > 0 && j < a.perm_full) {
        int64_t b, r, q2, r2;
        divmod(j, a.perm_f, a.perm_inv, b, r);
        divmod(r * a.perm_g, a.perm_f, a.perm_inv, q2, r2);
        return b * a.perm_f + r2;
    }
    return j;
}

__device__ __forceinline__ uint32_t mix32(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return (uint32_t)k;
}

// Insert (parent slot, face) into the open-addressing table of candidate
// prefixes; returns the slot, which identifies the face sequence.
__device__ int32_t cand_insert(uint64_t* table, uint64_t mask, int32_t parent, int32_t face, uint32_t* overflow) {
    const uint64_t key = ((uint64_t)(uint32_t)(parent + 1) << 32) | (uint32_t)face;
    uint64_t h = mix32(key) & mask;
    for (int probe = 0; probe < 256; ++probe) {
        uint64_t cur = __hip_atomic_load(table + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == key) return (int32_t)h;
        if (cur == kEmptyKey) {
            uint64_t prev = atomicCAS((unsigned long long*)(table + h), (unsigned long long)kEmptyKey,
                                      (unsigned long long)key);
            if (prev == kEmptyKey || prev == key) return (int32_t)h;
        }
        h = (h + 1) & mask;
    }
    atomicOr(overflow, 1u);
    return -2;
}

// Ray state in registers; loaded from / stored to the 96-byte queue record
// with 16-byte vector accesses.  In reception-sphere mode (SPH) the prefix
// word holds the path length so far and the last 16 bytes the face sequence.
struct Ray {
    d3 o, d;
    float E[6];
    int32_t excl, prefix, ray;
    float s;          // SPH: path length before the current segment [m]
    uint32_t seq[4];  // SPH: faces of the reflections so far, 24 bits each
};

template <bool SPH>
__device__ __forceinline__ void load_ray(const RayState* __restrict__ p, Ray& r) {
    const double2* q = reinterpret_cast<const double2*>(p);
    const double2 a0 = q[0], a1 = q[1], a2 = q[2];
    const float4 f0 = reinterpret_cast<const float4*>(p)[3];
    const int4 f1 = reinterpret_cast<const int4*>(p)[4];
    const int4 f2 = reinterpret_cast<const int4*>(p)[5];
    r.o = d3{a0.x, a0.y, a1.x};
    r.d = d3{a1.y, a2.x, a2.y};
    r.E[0] = f0.x;
    r.E[1] = f0.y;
    r.E[2] = f0.z;
    r.E[3] = f0.w;
    r.E[4] = __int_as_float(f1.x);
    r.E[5] = __int_as_float(f1.y);
    r.excl = f1.z;
    if (SPH) {
        r.prefix = -1;
        r.s = __int_as_float(f1.w);
        r.ray = -1;
        r.seq[0] = (uint32_t)f2.x;
        r.seq[1] = (uint32_t)f2.y;
        r.seq[2] = (uint32_t)f2.z;
        r.seq[3] = (uint32_t)f2.w;
    } else {
        r.prefix = f1.w;
        r.ray = f2.x;
    }
}

template <bool SPH>
__device__ __forceinline__ void store_ray(RayState* __restrict__ p, const Ray& r) {
    double2* q = reinterpret_cast<double2*>(p);
    q[0] = double2{r.o.x, r.o.y};
    q[1] = double2{r.o.z, r.d.x};
    q[2] = double2{r.d.y, r.d.z};
    reinterpret_cast<float4*>(p)[3] = float4{r.E[0], r.E[1], r.E[2], r.E[3]};
    if (SPH) {
        reinterpret_cast<int4*>(p)[4] = int4{__float_as_int(r.E[4]), __float_as_int(r.E[5]), r.excl, __float_as_int(r.s)};
        reinterpret_cast<int4*>(p)[5] = int4{(int)r.seq[0], (int)r.seq[1], (int)r.seq[2], (int)r.seq[3]};
    } else {
        reinterpret_cast<int4*>(p)[4] = int4{__float_as_int(r.E[4]), __float_as_int(r.E[5]), r.excl, r.prefix};
        reinterpret_cast<int4*>(p)[5] = int4{r.ray, 0, 0, 0};
    }
}

// Face i (0..4) of a packed sequence: bits [24 i, 24 i + 24) of the 128-bit
// little-endian word seq (constant word indices, so the array stays in registers).
__device__ __forceinline__ uint32_t get_face(const uint32_t seq[4], int i) {
    switch (i) {
        case 0: return seq[0] & 0xFFFFFFu;
        case 1: return ((seq[0] >> 24) | (seq[1] << 8)) & 0xFFFFFFu;
        case 2: return ((seq[1] >> 16) | (seq[2] << 16)) & 0xFFFFFFu;
        case 3: return (seq[2] >> 8) & 0xFFFFFFu;
        default: return seq[3] & 0xFFFFFFu;
    }
}

__device__ __forceinline__ void put_face(uint32_t seq[4], int i, uint32_t f) {
    switch (i) {
        case 0: seq[0] |= f; break;
        case 1: seq[0] |= f << 24; seq[1] |= f >> 8; break;
        case 2: seq[1] |= f << 16; seq[2] |= f >> 16; break;
        case 3: seq[2] |= f << 8; break;
        default: seq[3] |= f; break;
    }
}

// Insert (receiver, prefix slot) into the pair set.
__device__ void pair_insert(const SbrArgs& a, int32_t r, int32_t slot) {
    const uint64_t key = ((uint64_t)(uint32_t)r << 32) | (uint32_t)slot;
    uint64_t h = mix32(key ^ 0x5bd1e995ull) & a.pairs_mask;
    for (int probe = 0; probe < 256; ++probe) {
        const uint64_t cur = __hip_atomic_load(a.pairs + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == key) return;
        if (cur == kEmptyKey) {
            const uint64_t prev = atomicCAS((unsigned long long*)(a.pairs + h), (unsigned long long)kEmptyKey,
                                            (unsigned long long)key);
            if (prev == kEmptyKey || prev == key) return;
        }
        h = (h + 1) & a.pairs_mask;
    }
    atomicOr(a.pairs_overflow, 1u);
}

// Receivers whose reception sphere the segment o + t d, 0 <= t <= tbest
// (tbest = inf: no hit) passes: the closest approach t* = clamp((R - o) . d,
// 0, tbest) lies within sphere_k (s + t*) of R.  The segment is clipped to
// the receivers' height band and grid rectangle and walked cell by cell (2-D
// DDA); the face sequence's prefix slot is inserted on the first pair.
__device__ void sphere_pairs(const SbrArgs& a, const Ray& st, d3 o, d3 d, double tbest) {
    double t0 = 0.0, t1 = tbest;
    auto clip = [&](double oc, double dc, double lo, double hi) {
        if (dc != 0.0) {
            const double ta = (lo - oc) / dc, tb = (hi - oc) / dc;
            t0 = fmax(t0, fmin(ta, tb));
            t1 = fmin(t1, fmax(ta, tb));
        } else if (oc < lo || oc > hi) {
            t1 = -1.0;
        }
    };
    clip(o.z, d.z, a.rz_lo, a.rz_hi);
    clip(o.x, d.x, a.rgx0, a.rgx0 + a.rgnx * a.rgcell);
    clip(o.y, d.y, a.rgy0, a.rgy0 + a.rgny * a.rgcell);
    if (!(t0 <= t1)) return;
    const double px = o.x + t0 * d.x - a.rgx0, py = o.y + t0 * d.y - a.rgy0;
    int ix = min(max((int)floor(px / a.rgcell), 0), a.rgnx - 1);
    int iy = min(max((int)floor(py / a.rgcell), 0), a.rgny - 1);
    const int sx = d.x > 0.0 ? 1 : -1, sy = d.y > 0.0 ? 1 : -1;
    double tnx = d.x != 0.0 ? (a.rgx0 + (ix + (d.x > 0.0 ? 1 : 0)) * a.rgcell - o.x) / d.x : __builtin_inf();
    double tny = d.y != 0.0 ? (a.rgy0 + (iy + (d.y > 0.0 ? 1 : 0)) * a.rgcell - o.y) / d.y : __builtin_inf();
    const double dtx = d.x != 0.0 ? a.rgcell / fabs(d.x) : __builtin_inf();
    const double dty = d.y != 0.0 ? a.rgcell / fabs(d.y) : __builtin_inf();
    int32_t slot = -3;  // not looked up yet
    for (int it = 0; it < a.rgnx + a.rgny + 2; ++it) {
        const int c = iy * a.rgnx + ix;
        for (int j = a.cell_start[c]; j < a.cell_start[c + 1]; ++j) {
            const int32_t r = a.cell_rx[j];
            const d3 R{a.rx[3 * r], a.rx[3 * r + 1], a.rx[3 * r + 2]};
            double ts = dot(sub(R, o), d);
            ts = ts < 0.0 ? 0.0 : (ts > tbest ? tbest : ts);
            const d3 w = sub(add(o, scale(d, ts)), R);
            const double rad = a.sphere_k * ((double)st.s + ts);
            if (dot(w, w) <= rad * rad) {
                if (slot == -3) {
                    slot = -1;
                    for (int i = 0; i < a.depth && slot != -2; ++i)
                        slot = cand_insert(a.table, a.table_mask, slot, (int32_t)get_face(st.seq, i), a.overflow);
                }
                if (slot >= 0) pair_insert(a, r, slot);
            }
        }
        if (fmin(tnx, tny) > t1) break;
        if (tnx < tny) {
            ix += sx;
            tnx += dtx;
            if (ix < 0 || ix >= a.rgnx) break;
        } else {
            iy += sy;
            tny += dty;
            if (iy < 0 || iy >= a.rgny) break;
        }
    }
}

// Whether the ray o + t d, t > 0, crosses the coverage plane z = gz inside
// the grid; tc is the crossing's ray parameter.
__device__ __forceinline__ bool crosses_grid(const SbrArgs& a, d3 o, d3 d, double& tc) {
    if (!(fabs(d.z) >= 1e-12)) return false;
    tc = (a.gz - o.z) / d.z;
    if (!(tc > 0.0)) return false;
    const double x = o.x + tc * d.x, y = o.y + tc * d.y;
    const double fx = floor((x - a.gx0) / a.gcell), fy = floor((y - a.gy0) / a.gcell);
    return fx >= 0.0 && fx < (double)a.gnx && fy >= 0.0 && fy < (double)a.gny;
}

// Whether the ray o + t d, t >= 0, enters the receivers' height band and grid
// rectangle (the region where reception spheres are looked up).
__device__ __forceinline__ bool reaches_rx_region(const SbrArgs& a, d3 o, d3 d) {
    double t0 = 0.0, t1 = __builtin_inf();
    auto clip = [&](double oc, double dc, double lo, double hi) {
        if (dc != 0.0) {
            const double ta = (lo - oc) / dc, tb = (hi - oc) / dc;
            t0 = fmax(t0, fmin(ta, tb));
            t1 = fmin(t1, fmax(ta, tb));
        } else if (oc < lo || oc > hi) {
            t1 = -1.0;
        }
    };
    clip(o.z, d.z, a.rz_lo, a.rz_hi);
    clip(o.x, d.x, a.rgx0, a.rgx0 + a.rgnx * a.rgcell);
    clip(o.y, d.y, a.rgy0, a.rgy0 + a.rgny * a.rgcell);
    return t0 <= t1;
}

template <int MODE, bool FIRST, bool OVF>
#ifndef RT_TRACE_WAVES_PER_EU
#define RT_TRACE_WAVES_PER_EU 4
#endif
__global__ __launch_bounds__(kTraceBlock) __attribute__((amdgpu_waves_per_eu(RT_TRACE_WAVES_PER_EU)))
void sbr_bounce(SbrArgs a, MatTable mats) {
    __shared__ int32_t stack[kStack][kTraceBlock];
    __shared__ Node lds_nodes[kLdsNodes];
    const int n_lds = stage_nodes(a.sc, lds_nodes);
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * kTraceBlock + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * kTraceBlock) >> 6;
    // input regions: lane r of every wave holds the inclusive prefix of the
    // region counts up to r (registers, so no LDS is taken from the stack)
    uint32_t incl = 0;
    if (!FIRST) {
        incl = a.in_count[lane * kCounterStride];
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t v = __shfl_up(incl, off);
            if (lane >= off) incl += v;
        }
    }
    const int64_t count = FIRST ? a.chunk : (int64_t)__shfl(incl, 63);
    if (a.stats && blockIdx.x < 1 && threadIdx.x < 64) {
        // rays of this depth: the queue plus those dropped before a last bounce
        uint32_t dropped = FIRST ? 0u : a.in_count[lane * kCounterStride + 1];
        for (int off = 32; off >= 1; off >>= 1) dropped += __shfl_xor(dropped, off);
        if (threadIdx.x == 0) atomicAdd((unsigned long long*)&a.stats[a.depth], (unsigned long long)(count + dropped));
    }
    uint32_t wave_dropped = 0;  // rays of this wave dropped before the last bounce
    for (int64_t base = wave * 64; base < count; base += nwaves * 64) {
        const int64_t item = base + lane;
        const bool active = item < count;
        // region of item: the number of regions whose inclusive prefix is <= item
        // (a branch-free binary search over the lanes, taken by the whole wave)
        int region_in = 0;
        int64_t region_off = 0;
        if (!FIRST) {
            for (int s = 32; s >= 1; s >>= 1) {
                const uint32_t v = __shfl(incl, region_in + s - 1);
                if ((int64_t)v <= item) region_in += s;
            }
            const uint32_t prev = __shfl(incl, region_in > 0 ? region_in - 1 : 0);
            const uint32_t start = region_in > 0 ? prev : 0u;
            region_off = item - (int64_t)start;
        }
        Ray st;
        bool alive = false, dropped = false;
        if (active) {
            if (FIRST) {
                const int64_t pos = lattice_position(a, a.pos0 + item);
                st.d = fib_dir(a.begin + pos * a.stride, a.num_rays);
                st.o = d3{a.tx[0], a.tx[1], a.tx[2]};
                const f3 F = antenna_field(a.tx_ant, f3{(float)st.d.x, (float)st.d.y, (float)st.d.z});
                st.E[0] = F.x;
                st.E[1] = 0.0f;
                st.E[2] = F.y;
                st.E[3] = 0.0f;
                st.E[4] = F.z;
                st.E[5] = 0.0f;
                st.excl = -1;
                st.prefix = -1;
                st.ray = (int32_t)pos;
                st.s = 0.0f;
                st.seq[0] = st.seq[1] = st.seq[2] = st.seq[3] = 0u;
            } else {
                load_ray<(MODE & kModeSphere) != 0>(a.in + region_in * a.region_cap + region_off, st);
            }
            const d3 o = st.o;
            const d3 d = st.d;
            double tbest = __builtin_inf();
            TravStats ts;
            // The last bounce of a coverage map only deposits: its segment
            // matters up to the coverage plane, so it is searched only up to
            // there, and only until a first hit (any hit at t <= tc blocks the
            // deposit, exactly as the closest hit would); rays that do not cross
            // the plane inside the grid are not searched at all.
            bool search = true;
            const bool last = !FIRST && (MODE & kModeCoverage) && a.depth == a.max_depth;
            if (last) {
                double tc;
                search = crosses_grid(a, o, d, tc);
                if (search) tbest = __longlong_as_double(__double_as_longlong(tc) + 1);  // next double above tc
            }
            // in reception-sphere mode the last segment only meets spheres: one
            // that never enters the receivers' region needs no search
            if ((MODE & kModeSphere) && !FIRST && a.depth == a.max_depth) search = reaches_rx_region(a, o, d);
            int best = -1;
            if (last) {
                if (search)
                    best = traverse<false, (MODE & kModeStats) != 0, kTraceBlock, OVF, true>(
                        a.sc, lds_nodes, n_lds, o, d, st.excl, st.excl, a.tmin, tbest, stack, &ts);
            } else if (search) {
                best = traverse<false, (MODE & kModeStats) != 0, kTraceBlock, OVF>(
                    a.sc, lds_nodes, n_lds, o, d, st.excl, st.excl, a.tmin, tbest, stack, &ts);
            }
            if (MODE & kModeStats) {
                const int nd = a.max_depth + 1;
                atomicAdd((unsigned long long*)&a.work[a.depth], 1ull);
                atomicAdd((unsigned long long*)&a.work[nd + a.depth], (unsigned long long)ts.nodes);
                atomicAdd((unsigned long long*)&a.work[2 * nd + a.depth], (unsigned long long)ts.boxes);
                atomicAdd((unsigned long long*)&a.work[3 * nd + a.depth], (unsigned long long)ts.tris);
            }
            if ((MODE & kModeSphere) && a.depth >= 1) sphere_pairs(a, st, o, d, tbest);
            if (MODE & kModeRecord) {
                const int64_t at = (int64_t)a.depth * a.count + st.ray;
                a.rec_tri[at] = best >= 0 ? a.sc.tris[best].orig : -1;
                a.rec_t[at] = tbest;
            }
            if (MODE & kModeCoverage) {
                const double dz = d.z;
                if (fabs(dz) >= 1e-12) {
                    const double tc = (a.gz - o.z) / dz;
                    if (tc > 0.0 && tc < tbest) {
                        const double x = o.x + tc * d.x, y = o.y + tc * d.y;
                        const double fx = floor((x - a.gx0) / a.gcell), fy = floor((y - a.gy0) / a.gcell);
                        if (fx >= 0.0 && fx < (double)a.gnx && fy >= 0.0 && fy < (double)a.gny) {
                            const f3 fr = antenna_field(a.rx_ant, f3{(float)-d.x, (float)-d.y, (float)-d.z});
                            const float ar = fr.x * st.E[0] + fr.y * st.E[2] + fr.z * st.E[4];
                            const float ai = fr.x * st.E[1] + fr.y * st.E[3] + fr.z * st.E[5];
                            const float w = a.wscale * (ar * ar + ai * ai) / fabsf((float)dz);
                            const int64_t cell = (int64_t)fy * a.gnx + (int64_t)fx;
                            atomicAdd(a.gain + cell, w);
                            atomicAdd(a.hits + cell, 1u);
                        }
                    }
                }
            }
            if (best >= 0 && a.depth < a.max_depth) {
                alive = true;
                const Shade sh = a.sc.shades[best];
                // the material's fields in one round trip to memory (used here, so
                // that no load is sunk into the branches below)
                Mat mt{};
                mt.eta_re = mats.m[sh.mat].eta_re;
                mt.eta_im = mats.m[sh.mat].eta_im;
                mt.pec = mats.m[sh.mat].pec;
                mt.scat = mats.m[sh.mat].scat;
                asm volatile("" ::"v"(mt.eta_re), "v"(mt.eta_im), "v"(mt.pec), "v"(mt.scat));
                d3 n{sh.n[0], sh.n[1], sh.n[2]};
                if (dot(d, n) > 0.0) n = scale(n, -1.0);
                const double cos_i = -dot(d, n);
                const d3 dr = add(d, scale(n, 2.0 * cos_i));
                const d3 p = add(o, scale(d, tbest));
                const d3 ep = perp_basis(d, n);
                const d3 eli = cross(ep, d);
                const d3 elr = cross(ep, dr);
                cf rp, rl;
                fresnel(mt, (float)cos_i, rp, rl);
                const f3 fep{(float)ep.x, (float)ep.y, (float)ep.z};
                const f3 feli{(float)eli.x, (float)eli.y, (float)eli.z};
                f3 felr{(float)elr.x, (float)elr.y, (float)elr.z};
                // diffuse scattering (coverage and record modes): with probability
                // S^2 the ray leaves in a Lambertian direction and the reflected
                // components ride on that direction's transverse basis
                d3 dout = dr;
                f3 fepo = fep;
                if ((MODE & (kModeCoverage | kModeRecord)) && mt.scat > 0.0f) {
                    const uint64_t ri = (uint64_t)(a.begin + (int64_t)st.ray * a.stride);
                    const uint64_t c0 = (ri * (uint64_t)(a.max_depth + 1) + (uint64_t)a.depth) * 3ull;
                    const double S = (double)mt.scat;
                    if (uniform01(a.scat_seed, c0) < S * S) {
                        dout = lambert_dir(n, uniform01(a.scat_seed, c0 + 1), uniform01(a.scat_seed, c0 + 2));
                        const d3 eps = perp_basis(dout, n);
                        const d3 els = cross(eps, dout);
                        fepo = f3{(float)eps.x, (float)eps.y, (float)eps.z};
                        felr = f3{(float)els.x, (float)els.y, (float)els.z};
                    }
                }
                const cf Ex{st.E[0], st.E[1]}, Ey{st.E[2], st.E[3]}, Ez{st.E[4], st.E[5]};
                const cf ap{fep.x * Ex.re + fep.y * Ey.re + fep.z * Ez.re, fep.x * Ex.im + fep.y * Ey.im + fep.z * Ez.im};
                const cf al{feli.x * Ex.re + feli.y * Ey.re + feli.z * Ez.re,
                            feli.x * Ex.im + feli.y * Ey.im + feli.z * Ez.im};
                const cf sp = cmul(rp, ap), sl = cmul(rl, al);
                st.E[0] = sp.re * fepo.x + sl.re * felr.x;
                st.E[1] = sp.im * fepo.x + sl.im * felr.x;
                st.E[2] = sp.re * fepo.y + sl.re * felr.y;
                st.E[3] = sp.im * fepo.y + sl.im * felr.y;
                st.E[4] = sp.re * fepo.z + sl.re * felr.z;
                st.E[5] = sp.im * fepo.z + sl.im * felr.z;
                st.o = p;
                st.d = dout;
                st.excl = sh.face;
                // a ray entering the last bounce of a map only deposits there: one
                // that cannot cross the coverage plane inside the grid is dropped
                // here (and still counted as a ray of that depth)
                if ((MODE & ~kModeStats) == kModeCoverage && a.depth + 1 == a.max_depth) {
                    double tc;
                    if (!crosses_grid(a, p, dout, tc)) {
                        alive = false;
                        dropped = true;
                    }
                }
                // likewise in reception-sphere mode for a last segment that cannot
                // enter the receivers' region
                if (MODE == kModeSphere && a.depth + 1 == a.max_depth && !reaches_rx_region(a, p, dout)) {
                    alive = false;
                    dropped = true;
                }
                if (MODE & kModeCandidates) {
                    if (st.prefix != -2) st.prefix = cand_insert(a.table, a.table_mask, st.prefix, sh.face, a.overflow);
                }
                if (MODE & kModeSphere) {
                    st.s += (float)tbest;
                    put_face(st.seq, a.depth, (uint32_t)sh.face);
                }
            }
        }
        if ((MODE & ~kModeStats) == kModeCoverage || MODE == kModeSphere)
            wave_dropped += (uint32_t)__popcll(__ballot(dropped));
        // wave-ballot compaction of the survivors into the next queue
        const uint64_t m = __ballot(alive);
        if (m) {
            uint32_t b = 0;
            const int region = (int)(wave % kQueueRegions);
            if (lane == 0) b = atomicAdd(a.out_count + region * kCounterStride, (uint32_t)__popcll(m));
            b = __shfl(b, 0);
            if (alive)
                store_ray<(MODE & kModeSphere) != 0>(
                    a.out + region * a.region_cap + b + __popcll(m & ((1ull << lane) - 1ull)), st);
        }
    }
    // the dropped rays go to word 1 of the region counter (the next launch adds
    // them to its ray count)
    if (lane == 0 && wave_dropped) atomicAdd(a.out_count + (wave % kQueueRegions) * kCounterStride + 1, wave_dropped);
}

__global__ void fib_dirs_kernel(int64_t N, int64_t begin, int64_t stride, int64_t count, double* out) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    d3 d = fib_dir(begin + j * stride, N);
    out[3 * j] = d.x;
    out[3 * j + 1] = d.y;
    out[3 * j + 2] = d.z;
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void finalize_db_kernel(const float* __restrict__ g, float* __restrict__ db, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = g[i];
    db[i] = v > 0.0f ? 10.0f * log10f(v) : -__builtin_inff();
}

template <int MODE, bool OVF>
void launch_depth(const SbrArgs& a, const MatTable& mats, int grid, hipStream_t s) {
    if (a.depth == 0)
        hipLaunchKernelGGL((sbr_bounce<MODE, true, OVF>), dim3(grid), dim3(kTraceBlock), 0, s, a, mats);
    else
        hipLaunchKernelGGL((sbr_bounce<MODE, false, OVF>), dim3(grid), dim3(kTraceBlock), 0, s, a, mats);
}

template <int MODE>
hipError_t launch_mode(const SbrArgs& a, const MatTable& mats, int grid, hipStream_t s) {
    if (a.sc.stack_need > kStack) launch_depth<MODE, true>(a, mats, grid, s);
    else launch_depth<MODE, false>(a, mats, grid, s);
    return hipGetLastError();
}

}  // namespace

int64_t sbr_region_capacity(int64_t chunk, int grid) {
    const int64_t nwaves = (int64_t)grid * (kTraceBlock / 64);
    const int64_t iters = (chunk + nwaves * 64 - 1) / (nwaves * 64);
    return ((nwaves + kQueueRegions - 1) / kQueueRegions) * iters * 64;
}

hipError_t launch_sbr_bounce(const SbrArgs& a, const MatTable& mats, int mode, int grid, hipStream_t s) {
    switch (mode) {
        case kModeCoverage: return launch_mode<kModeCoverage>(a, mats, grid, s);
        case kModeRecord: return launch_mode<kModeRecord>(a, mats, grid, s);
        case kModeCandidates: return launch_mode<kModeCandidates>(a, mats, grid, s);
        case kModeSphere: return launch_mode<kModeSphere>(a, mats, grid, s);
        case kModeCoverage | kModeStats: return launch_mode<kModeCoverage | kModeStats>(a, mats, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fib_dirs(int64_t N, int64_t begin, int64_t stride, int64_t count, double* out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(fib_dirs_kernel, dim3((unsigned)blocks), dim3(256), 0, s, N, begin, stride, count, out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(void* p, uint32_t v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t blocks = ((int64_t)n + 255) / 256;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, v, (int64_t)n);
    return hipGetLastError();
}

hipError_t launch_finalize_db(const float* gain, float* db, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(finalize_db_kernel, dim3((unsigned)blocks), dim3(256), 0, s, gain, db, n);
    return hipGetLastError();
}

}  // namespace rt
