// C ABI of the gfx950 radio ray tracer (declared in include/rt.h): context
// and scene handles, host-side argument validation, scratch management and
// the launch sequences of the coverage, path and gradient computations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rt.h"
#include "kernels.h"
#include "scene.h"

namespace {

thread_local std::string g_err;

rt_status fail(rt_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define RT_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(e_ == hipErrorOutOfMemory ? RT_ERR_OOM : RT_ERR_DEVICE,                        \
                        std::string(#call) + ": " + hipGetErrorString(e_));                            \
    } while (0)

constexpr double kEps0 = 8.8541878128e-12;
constexpr double kC0 = 299792458.0;
// Rays per launch sequence.  The two ray queues of a chunk take 2 x 12.9 GB at
// 2^27 rays (a 1e8-ray lattice in one sequence of max_depth + 1 launches).
constexpr int64_t kChunk = int64_t(1) << 27;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

hipError_t ensure(DevBuf& b, size_t bytes) {
    if (b.bytes >= bytes) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess) return e;
    }
    b.p = nullptr;
    b.bytes = 0;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipSuccess) b.bytes = bytes;
    return e;
}

// Scratch of rt_coverage_map_noalloc: the two ray queues and the queue-region
// counters of the shoot-and-bounce launches, in a file-scope device array (one
// copy per GPU, alive until the process ends).  Host code uses only the
// addresses hipGetSymbolAddress returns for it, never the array's name.
constexpr size_t kNoAllocCounterBytes = 64 << 10;
static_assert(9 * rt::kQueueRegions * rt::kCounterStride * sizeof(uint32_t) <= kNoAllocCounterBytes,
              "queue counters of nine depths must fit the fixed scratch");
constexpr size_t kNoAllocScratchBytes = (size_t(112) << 20) + kNoAllocCounterBytes;
constexpr int64_t kNoAllocMaxChunk = int64_t(1) << 19;  // rays per launch sequence
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `device` (looked up once
// per device).
rt_status scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return fail(RT_ERR_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(RT_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return RT_OK;
}

// Fixed queue memory handed to run_sbr instead of the context's buffers.
struct FixedQueues {
    rt::RayState* q[2];
    uint32_t* counters;
    int64_t max_chunk;
};

}  // namespace

struct rt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    DevBuf queue[2];
    DevBuf counters;   // uint32 [depth + 1][kQueueRegions][kCounterStride] queue region counts
    DevBuf table;      // candidate prefix table
    DevBuf pairs;      // reception-sphere (receiver, prefix slot) set
    DevBuf pair_rx;    // receiver of each extracted pair
    DevBuf rgrid;      // receiver grid: cell starts then receiver lists
    DevBuf cands;
    DevBuf rx;         // double [nrx][3]
    DevBuf rx_ant;     // Antenna [nrx]
    DevBuf paths;      // unsorted path records
    DevBuf chan;       // channel responses: element offsets and velocities
    DevBuf scat;       // scattered paths: points, masks, prefixes, counts of one chunk
    void* scratch = nullptr;  // this device's copy of the fixed scratch array
    int64_t last_candidates = 0;
    // launch timing of the shoot-and-bounce kernels
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    struct Rec {
        int depth;
        hipEvent_t start, stop;
    };
    std::vector<Rec> recs;
    size_t ev_used = 0;
};

struct rt_scene {
    rt_ctx* ctx = nullptr;
    rt::HostScene host;
    std::vector<rt_material> mats;
    std::vector<float> scat;   // scattering coefficient per material (empty: none)
    uint64_t scat_seed = 0;
    DevBuf nodes, tris, shades, faces, face_tris, leaf_of_input, wedges;
    rt::DevScene dev{};
};

namespace {

bool finite3(const float* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

rt_status check_device(const rt_device* d, const char* what, double max_abs) {
    if (!d) return fail(RT_ERR_ARG, std::string(what) + " is NULL");
    if (!finite3(d->pos) || !std::isfinite(d->yaw) || !std::isfinite(d->pitch) || !std::isfinite(d->roll))
        return fail(RT_ERR_ARG, std::string(what) + " has a non-finite position or orientation");
    if (d->pattern != RT_PATTERN_ISO && d->pattern != RT_PATTERN_TR38901 && d->pattern != RT_PATTERN_DIPOLE)
        return fail(RT_ERR_ARG, std::string(what) + " has an unknown antenna pattern");
    if (d->pol < RT_POL_V || d->pol > RT_POL_SLANT_M45)
        return fail(RT_ERR_ARG, std::string(what) + " has an unknown polarisation");
    if (max_abs > 0)
        for (int i = 0; i < 3; ++i)
            if (std::fabs(d->pos[i]) > 4.0 * max_abs)
                return fail(RT_ERR_ARG, std::string(what) + " lies more than 4x the scene extent from the origin");
    return RT_OK;
}

rt_status check_params(const rt_trace_params* p) {
    if (!p) return fail(RT_ERR_ARG, "params is NULL");
    if (!(p->freq_hz > 0) || !std::isfinite(p->freq_hz)) return fail(RT_ERR_ARG, "freq_hz must be positive");
    if (p->max_depth < 0 || p->max_depth > 8) return fail(RT_ERR_ARG, "max_depth must be in [0, 8]");
    if (p->num_rays < 1 || p->num_rays > (int64_t(1) << 40)) return fail(RT_ERR_ARG, "num_rays must be in [1, 2^40]");
    if (!(p->t_min >= 0) || !std::isfinite(p->t_min)) return fail(RT_ERR_ARG, "t_min must be finite and >= 0");
    if (p->ray_begin < 0 || p->ray_begin >= p->num_rays) return fail(RT_ERR_ARG, "ray_begin must be in [0, N)");
    if (p->ray_stride < 1) return fail(RT_ERR_ARG, "ray_stride must be >= 1");
    int64_t count = (p->num_rays - p->ray_begin + p->ray_stride - 1) / p->ray_stride;
    if (count >= (int64_t(1) << 31)) return fail(RT_ERR_ARG, "more than 2^31 - 1 traced rays per call");
    if (p->cand_mode != RT_CAND_ALL && p->cand_mode != RT_CAND_SPHERE)
        return fail(RT_ERR_ARG, "cand_mode must be RT_CAND_ALL or RT_CAND_SPHERE");
    if (p->cand_mode == RT_CAND_SPHERE && (!(p->sphere_kappa > 0) || !std::isfinite(p->sphere_kappa)))
        return fail(RT_ERR_ARG, "sphere_kappa must be positive");
    return RT_OK;
}

int64_t traced_count(const rt_trace_params* p) {
    return (p->num_rays - p->ray_begin + p->ray_stride - 1) / p->ray_stride;
}

void rot(double yaw, double pitch, double roll, double R[9]) {
    double cy = std::cos(yaw), sy = std::sin(yaw), cp = std::cos(pitch), sp = std::sin(pitch);
    double cr = std::cos(roll), sr = std::sin(roll);
    // Rz(yaw) Ry(pitch) Rx(roll)
    R[0] = cy * cp; R[1] = cy * sp * sr - sy * cr; R[2] = cy * sp * cr + sy * sr;
    R[3] = sy * cp; R[4] = sy * sp * sr + cy * cr; R[5] = sy * sp * cr - cy * sr;
    R[6] = -sp;     R[7] = cp * sr;                R[8] = cp * cr;
}

rt::Antenna make_antenna(const rt_device* d) {
    rt::Antenna a{};
    rot(d->yaw, d->pitch, d->roll, a.Rd);
    for (int i = 0; i < 9; ++i) a.R[i] = (float)a.Rd[i];
    a.pattern = d->pattern;
    a.pol = d->pol;
    return a;
}

rt::MatTable make_mats(const rt_scene* s, double freq) {
    rt::MatTable t{};
    const double w = 2.0 * M_PI * freq;
    for (size_t i = 0; i < s->mats.size(); ++i) {
        rt::Mat& m = t.m[i];
        const double er = s->mats[i].eps_r, sg = s->mats[i].sigma;
        m.pec = std::isinf(sg) ? 1 : 0;
        m.eta_re_d = er;
        m.eta_im_d = m.pec ? 0.0 : -sg / (kEps0 * w);
        m.eta_re = (float)m.eta_re_d;
        m.eta_im = (float)m.eta_im_d;
        m.scat = i < s->scat.size() ? s->scat[i] : 0.0f;
    }
    return t;
}

rt_status check_materials(const rt_material* mats, int32_t nm) {
    if (!mats || nm < 1 || nm > rt::kMaxMaterials)
        return fail(RT_ERR_ARG, "number of materials must be in [1, " + std::to_string(rt::kMaxMaterials) + "]");
    for (int32_t i = 0; i < nm; ++i) {
        if (!(mats[i].eps_r > 0) || !std::isfinite(mats[i].eps_r))
            return fail(RT_ERR_ARG, "material " + std::to_string(i) + ": eps_r must be finite and positive");
        if (!(mats[i].sigma >= 0) || std::isnan(mats[i].sigma))
            return fail(RT_ERR_ARG, "material " + std::to_string(i) + ": sigma must be >= 0 (or +inf)");
    }
    return RT_OK;
}

// Band permutation for coherent ray order: F = largest Fibonacci number
// <= sqrt(64 pi count), G the one before it (0 disables).
void band_perm(int64_t count, int64_t stride, int64_t& F, int64_t& G) {
    F = G = 0;
    if (stride != 1 || count < 256) return;
    double target = std::sqrt(64.0 * M_PI * (double)count);
    int64_t a = 1, b = 2;
    while ((double)(a + b) <= target) {
        int64_t c = a + b;
        a = b;
        b = c;
    }
    F = b;
    G = a;
}

int grid_for(const rt_ctx* c) { return c->num_cu * 4; }
// Blocks of the shoot-and-bounce launch of depth k when the queues are
// allocated per call (measured on the large city: more, smaller blocks for the
// coherent first bounce, fewer for the second), and the region capacity that
// covers every such grid.  The fixed-scratch path keeps grid_for for all
// depths: a larger grid's minimum region capacity would not fit its scratch.
int grid_for_depth(const rt_ctx* c, int k) { return c->num_cu * (k == 0 ? 8 : k == 1 ? 2 : 4); }
int64_t region_capacity_by_depth(const rt_ctx* c, int64_t chunk) {
    int64_t cap = 0;
    for (int k = 0; k < 3; ++k) cap = std::max(cap, rt::sbr_region_capacity(chunk, grid_for_depth(c, k)));
    return cap;
}

// Runs the shoot-and-bounce launches for all rays of one transmitter.
rt_status run_sbr(rt_ctx* c, rt_scene* s, const rt_trace_params* p, const rt_device* tx, const rt_device* rx_ant,
                  const rt_grid* g, int mode, float* gain, uint32_t* hits, uint64_t* stats, int32_t* rec_tri,
                  double* rec_t, uint64_t* table, uint64_t table_mask, uint32_t* overflow,
                  uint64_t* work = nullptr, const rt::SbrArgs* sphere = nullptr, const FixedQueues* fixed = nullptr) {
    const int64_t count = traced_count(p);
    const int64_t chunk = std::min(count, fixed ? fixed->max_chunk : kChunk);
    const int64_t region_cap =
        fixed ? rt::sbr_region_capacity(chunk, grid_for(c)) : region_capacity_by_depth(c, chunk);
    rt::RayState* queue[2];
    uint32_t* cnt;
    if (fixed) {
        queue[0] = fixed->q[0];
        queue[1] = fixed->q[1];
        cnt = fixed->counters;
    } else {
        const size_t qbytes = (size_t)rt::kQueueRegions * region_cap * sizeof(rt::RayState);
        RT_HIP(ensure(c->queue[0], qbytes));
        RT_HIP(ensure(c->queue[1], qbytes));
        RT_HIP(ensure(c->counters, (size_t)(p->max_depth + 1) * rt::kQueueRegions * rt::kCounterStride * sizeof(uint32_t)));
        queue[0] = (rt::RayState*)c->queue[0].p;
        queue[1] = (rt::RayState*)c->queue[1].p;
        cnt = (uint32_t*)c->counters.p;
    }
    rt::MatTable mats = make_mats(s, p->freq_hz);
    rt::SbrArgs a{};
    a.sc = s->dev;
    a.num_rays = p->num_rays;
    a.begin = p->ray_begin;
    a.stride = p->ray_stride;
    a.count = count;
    band_perm(count, p->ray_stride, a.perm_f, a.perm_g);
    a.perm_full = a.perm_f ? (count / a.perm_f) * a.perm_f : 0;
    a.perm_inv = a.perm_f ? 1.0 / (double)a.perm_f : 0.0;
    a.tmin = p->t_min;
    a.scat_seed = s->scat_seed;
    for (int i = 0; i < 3; ++i) a.tx[i] = tx->pos[i];
    a.tx_ant = make_antenna(tx);
    if (rx_ant) a.rx_ant = make_antenna(rx_ant);
    if (g) {
        a.gx0 = g->x0;
        a.gy0 = g->y0;
        a.gcell = g->cell;
        a.gz = g->z;
        a.gnx = g->nx;
        a.gny = g->ny;
        const double lam = kC0 / p->freq_hz;
        a.wscale = (float)((lam / (4.0 * M_PI)) * (lam / (4.0 * M_PI)) * (4.0 * M_PI / (double)p->num_rays) /
                           (g->cell * g->cell));
    }
    a.gain = gain;
    a.hits = hits;
    a.max_depth = p->max_depth;
    a.stats = stats;
    a.work = work;
    a.rec_tri = rec_tri;
    a.rec_t = rec_t;
    a.table = table;
    a.table_mask = table_mask;
    a.overflow = overflow;
    if (sphere) {
        a.rx = sphere->rx;
        a.cell_start = sphere->cell_start;
        a.cell_rx = sphere->cell_rx;
        a.rgx0 = sphere->rgx0;
        a.rgy0 = sphere->rgy0;
        a.rgcell = sphere->rgcell;
        a.rgnx = sphere->rgnx;
        a.rgny = sphere->rgny;
        a.rz_lo = sphere->rz_lo;
        a.rz_hi = sphere->rz_hi;
        a.sphere_k = sphere->sphere_k;
        a.pairs = sphere->pairs;
        a.pairs_mask = sphere->pairs_mask;
        a.pairs_overflow = sphere->pairs_overflow;
    }
    const bool profiling = c->profiling && !fixed;  // the fixed-memory path creates no events
    for (int64_t pos0 = 0; pos0 < count; pos0 += chunk) {
        a.pos0 = pos0;
        a.chunk = std::min(chunk, count - pos0);
        const size_t nwords = (size_t)(p->max_depth + 1) * rt::kQueueRegions * rt::kCounterStride;
        if (fixed) RT_HIP(rt::launch_fill_u32(cnt, 0u, nwords, c->stream));
        else RT_HIP(hipMemsetAsync(cnt, 0, nwords * sizeof(uint32_t), c->stream));
        for (int k = 0; k <= p->max_depth; ++k) {
            a.depth = k;
            a.in = k ? queue[(k - 1) & 1] : nullptr;
            a.in_count = k ? cnt + (size_t)(k - 1) * rt::kQueueRegions * rt::kCounterStride : nullptr;
            a.out = queue[k & 1];
            a.out_count = cnt + (size_t)k * rt::kQueueRegions * rt::kCounterStride;
            a.region_cap = region_cap;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (profiling) {
                while (c->ev_pool.size() < c->ev_used + 2) {
                    hipEvent_t e;
                    RT_HIP(hipEventCreate(&e));
                    c->ev_pool.push_back(e);
                }
                e0 = c->ev_pool[c->ev_used++];
                e1 = c->ev_pool[c->ev_used++];
                RT_HIP(hipEventRecord(e0, c->stream));
            }
            RT_HIP(rt::launch_sbr_bounce(a, mats, mode, fixed ? grid_for(c) : grid_for_depth(c, k), c->stream));
            if (profiling) {
                RT_HIP(hipEventRecord(e1, c->stream));
                c->recs.push_back({k, e0, e1});
            }
        }
    }
    return RT_OK;
}

}  // namespace

// accessors used by the surrogate's C ABI (mlp_api.hip)
rt_status rt_internal_fail(rt_status code, const char* msg) { return fail(code, msg); }
hipStream_t rt_internal_stream(rt_ctx* c) { return c->stream; }
int rt_internal_device(rt_ctx* c) { return c->device; }
rt_ctx* rt_internal_scene_ctx(const rt_scene* s) { return s->ctx; }

extern "C" {

const char* rt_last_error(void) { return g_err.c_str(); }

rt_status rt_create(rt_ctx** out, int32_t device) {
    if (!out) return fail(RT_ERR_ARG, "out is NULL");
    int n = 0;
    RT_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(RT_ERR_ARG, "no such HIP device");
    RT_HIP(hipSetDevice(device));
    void* scr = nullptr;
    const rt_status st = scratch_address(device, &scr);
    if (st != RT_OK) return st;
    rt_ctx* c = new rt_ctx();
    c->device = device;
    c->scratch = scr;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0) c->num_cu = cu;
    *out = c;
    return RT_OK;
}

rt_status rt_destroy(rt_ctx* c) {
    if (!c) return RT_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (DevBuf* b : {&c->queue[0], &c->queue[1], &c->counters, &c->table, &c->cands, &c->rx, &c->rx_ant, &c->paths,
                      &c->pairs, &c->pair_rx, &c->rgrid, &c->chan, &c->scat})
        if (b->p) (void)hipFree(b->p);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
    return RT_OK;
}

rt_status rt_set_stream(rt_ctx* c, void* stream) {
    if (!c) return fail(RT_ERR_ARG, "ctx is NULL");
    c->stream = (hipStream_t)stream;
    return RT_OK;
}

rt_status rt_synchronize(rt_ctx* c) {
    if (!c) return fail(RT_ERR_ARG, "ctx is NULL");
    RT_HIP(hipSetDevice(c->device));
    RT_HIP(hipStreamSynchronize(c->stream));
    return RT_OK;
}

rt_status rt_scene_create(rt_ctx* c, const float* V, int64_t nv, const int32_t* F, int64_t nt,
                          const int32_t* tri_mat, const rt_material* mats, int32_t nm, rt_scene** out) {
    if (!c || !V || !F || !tri_mat || !out) return fail(RT_ERR_ARG, "NULL argument");
    if (nv < 3) return fail(RT_ERR_ARG, "need at least 3 vertices");
    rt_status st = check_materials(mats, nm);
    if (st != RT_OK) return st;
    rt_scene* s = new rt_scene();
    s->ctx = c;
    std::string err;
    if (rt::build_scene(V, nv, F, nt, tri_mat, nm, s->host, err) != 0) {
        delete s;
        return fail(RT_ERR_ARG, err);
    }
    s->mats.assign(mats, mats + nm);
    hipError_t e = hipSetDevice(c->device);
    auto up = [&](DevBuf& b, const void* src, size_t bytes) {
        if (e != hipSuccess) return;
        e = ensure(b, std::max<size_t>(bytes, 64));
        if (e == hipSuccess && bytes) e = hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice);
    };
    const rt::HostScene& h = s->host;
    up(s->nodes, h.nodes.data(), h.nodes.size() * sizeof(rt::Node));
    up(s->tris, h.tris.data(), h.tris.size() * sizeof(rt::Tri));
    up(s->shades, h.shades.data(), h.shades.size() * sizeof(rt::Shade));
    up(s->faces, h.faces.data(), h.faces.size() * sizeof(rt::Face));
    up(s->face_tris, h.face_tris.data(), h.face_tris.size() * sizeof(int32_t));
    std::vector<int32_t> leaf(h.tris.size());
    for (size_t k = 0; k < h.tris.size(); ++k) leaf[h.tris[k].orig] = (int32_t)k;
    up(s->leaf_of_input, leaf.data(), leaf.size() * sizeof(int32_t));
    up(s->wedges, h.wedges.data(), h.wedges.size() * sizeof(rt::Wedge));
    if (e != hipSuccess) {
        rt_scene_destroy(s);
        return fail(e == hipErrorOutOfMemory ? RT_ERR_OOM : RT_ERR_DEVICE, hipGetErrorString(e));
    }
    s->dev.nodes = (const rt::Node*)s->nodes.p;
    s->dev.tris = (const rt::Tri*)s->tris.p;
    s->dev.shades = (const rt::Shade*)s->shades.p;
    s->dev.faces = (const rt::Face*)s->faces.p;
    s->dev.face_tris = (const int32_t*)s->face_tris.p;
    s->dev.num_faces = h.num_faces;
    s->dev.nt = (int32_t)nt;
    s->dev.num_nodes = (int32_t)h.nodes.size();
    s->dev.stack_need = h.stack_need;
    s->dev.leaf_of_input = (const int32_t*)s->leaf_of_input.p;
    s->dev.wedges = (const rt::Wedge*)s->wedges.p;
    s->dev.num_wedges = (int32_t)h.wedges.size();
    *out = s;
    return RT_OK;
}

rt_status rt_scene_set_materials(rt_scene* s, const rt_material* mats, int32_t nm) {
    if (!s) return fail(RT_ERR_ARG, "scene is NULL");
    rt_status st = check_materials(mats, nm);
    if (st != RT_OK) return st;
    if ((size_t)nm != s->mats.size()) return fail(RT_ERR_ARG, "material count differs from the scene's");
    s->mats.assign(mats, mats + nm);
    return RT_OK;
}

rt_status rt_scene_set_scattering(rt_scene* s, const float* S, int32_t nm, uint64_t seed) {
    if (!s || !S) return fail(RT_ERR_ARG, "NULL argument");
    if ((size_t)nm != s->mats.size()) return fail(RT_ERR_ARG, "material count differs from the scene's");
    for (int32_t i = 0; i < nm; ++i)
        if (!(S[i] >= 0.0f && S[i] <= 1.0f)) return fail(RT_ERR_ARG, "scattering coefficients must lie in [0, 1]");
    s->scat.assign(S, S + nm);
    s->scat_seed = seed;
    return RT_OK;
}

rt_status rt_scene_info(const rt_scene* s, rt_scene_info_t* out) {
    if (!s || !out) return fail(RT_ERR_ARG, "NULL argument");
    out->num_triangles = (int64_t)s->host.tris.size();
    out->num_faces = s->host.num_faces;
    out->num_materials = (int32_t)s->mats.size();
    out->bvh_nodes = (int64_t)s->host.nodes.size();
    out->bvh_depth = s->host.depth;
    out->num_wedges = (int32_t)s->host.wedges.size();
    out->build_ms = s->host.build_ms;
    return RT_OK;
}

rt_status rt_scene_face_ids(const rt_scene* s, int32_t* ids) {
    if (!s || !ids) return fail(RT_ERR_ARG, "NULL argument");
    std::memcpy(ids, s->host.face_of_input.data(), s->host.face_of_input.size() * sizeof(int32_t));
    return RT_OK;
}

rt_status rt_scene_destroy(rt_scene* s) {
    if (!s) return RT_OK;
    if (s->ctx) (void)hipSetDevice(s->ctx->device);
    for (DevBuf* b : {&s->nodes, &s->tris, &s->shades, &s->faces, &s->face_tris, &s->leaf_of_input, &s->wedges})
        if (b->p) (void)hipFree(b->p);
    delete s;
    return RT_OK;
}

rt_status rt_fibonacci_directions(rt_ctx* c, int64_t N, int64_t begin, int64_t stride, int64_t count, double* dirs) {
    if (!c || (!dirs && count > 0)) return fail(RT_ERR_ARG, "NULL argument");
    if (N < 1 || begin < 0 || stride < 1 || count < 0) return fail(RT_ERR_ARG, "invalid lattice range");
    if (count > 0 && begin + (count - 1) * stride >= N) return fail(RT_ERR_ARG, "ray index beyond N");
    RT_HIP(hipSetDevice(c->device));
    RT_HIP(rt::launch_fib_dirs(N, begin, stride, count, dirs, c->stream));
    return RT_OK;
}

rt_status rt_trace_record(rt_ctx* c, rt_scene* s, const rt_trace_params* p, const rt_device* tx, int32_t* hit_tri,
                          double* hit_t) {
    if (!c || !s || !hit_tri || !hit_t) return fail(RT_ERR_ARG, "NULL argument");
    rt_status st = check_params(p);
    if (st != RT_OK) return st;
    if ((st = check_device(tx, "tx", s->host.max_abs)) != RT_OK) return st;
    RT_HIP(hipSetDevice(c->device));
    const int64_t n = traced_count(p) * (p->max_depth + 1);
    RT_HIP(hipMemsetD32Async((hipDeviceptr_t)hit_tri, (int)-2, (size_t)n, c->stream));
    RT_HIP(hipMemsetAsync(hit_t, 0xff, (size_t)n * sizeof(double), c->stream));  // NaN until written
    return run_sbr(c, s, p, tx, nullptr, nullptr, rt::kModeRecord, nullptr, nullptr, nullptr, hit_tri, hit_t,
                   nullptr, 0, nullptr);
}

namespace {
rt_status coverage_impl(rt_ctx* c, rt_scene* s, const rt_trace_params* p, const rt_device* tx,
                        const rt_device* rx_ant, const rt_grid* g, float* gain, uint32_t* hits, float* gain_db,
                        uint64_t* ray_bounces, uint64_t* work, const FixedQueues* fixed = nullptr) {
    if (!c || !s || !g || !gain || !hits) return fail(RT_ERR_ARG, "NULL argument");
    rt_status st = check_params(p);
    if (st != RT_OK) return st;
    if ((st = check_device(tx, "tx", s->host.max_abs)) != RT_OK) return st;
    if ((st = check_device(rx_ant, "rx_ant", 0)) != RT_OK) return st;
    if (g->nx < 1 || g->ny < 1 || (int64_t)g->nx * g->ny > (int64_t(1) << 31))
        return fail(RT_ERR_ARG, "grid size must be positive and below 2^31 cells");
    if (!(g->cell > 0) || !std::isfinite(g->cell) || !std::isfinite(g->x0) || !std::isfinite(g->y0) ||
        !std::isfinite(g->z))
        return fail(RT_ERR_ARG, "grid origin, cell size and height must be finite, cell > 0");
    RT_HIP(hipSetDevice(c->device));
    const int64_t cells = (int64_t)g->nx * g->ny;
    if (fixed) {  // fill kernels: callers of the fixed-memory path may capture it in a graph
        RT_HIP(rt::launch_fill_u32(gain, 0u, (size_t)cells, c->stream));
        RT_HIP(rt::launch_fill_u32(hits, 0u, (size_t)cells, c->stream));
        if (ray_bounces) RT_HIP(rt::launch_fill_u32(ray_bounces, 0u, (size_t)(p->max_depth + 1) * 2, c->stream));
    } else {
        RT_HIP(hipMemsetAsync(gain, 0, (size_t)cells * sizeof(float), c->stream));
        RT_HIP(hipMemsetAsync(hits, 0, (size_t)cells * sizeof(uint32_t), c->stream));
        if (ray_bounces)
            RT_HIP(hipMemsetAsync(ray_bounces, 0, (size_t)(p->max_depth + 1) * sizeof(uint64_t), c->stream));
        if (work) RT_HIP(hipMemsetAsync(work, 0, (size_t)4 * (p->max_depth + 1) * sizeof(uint64_t), c->stream));
    }
    st = run_sbr(c, s, p, tx, rx_ant, g, work ? (rt::kModeCoverage | rt::kModeStats) : rt::kModeCoverage, gain, hits,
                 ray_bounces, nullptr, nullptr, nullptr, 0, nullptr, work, nullptr, fixed);
    if (st != RT_OK) return st;
    if (gain_db) RT_HIP(rt::launch_finalize_db(gain, gain_db, cells, c->stream));
    return RT_OK;
}
}  // namespace

rt_status rt_coverage_map(rt_ctx* c, rt_scene* s, const rt_trace_params* p, const rt_device* tx,
                          const rt_device* rx_ant, const rt_grid* g, float* gain, uint32_t* hits, float* gain_db,
                          uint64_t* ray_bounces) {
    return coverage_impl(c, s, p, tx, rx_ant, g, gain, hits, gain_db, ray_bounces, nullptr);
}

rt_status rt_coverage_map_noalloc(rt_ctx* c, rt_scene* s, const rt_trace_params* p, const rt_device* tx,
                                  const rt_device* rx_ant, const rt_grid* g, float* gain, uint32_t* hits,
                                  float* gain_db, uint64_t* ray_bounces) {
    if (!c) return fail(RT_ERR_ARG, "ctx is NULL");
    if (!c->scratch) return fail(RT_ERR_DEVICE, "the context has no scratch address (rt_create did not set it)");
    if (p && (p->max_depth < 0 || p->max_depth > 8)) return fail(RT_ERR_ARG, "max_depth must be in [0, 8]");
    // queues of the largest chunk whose two queues fit the scratch beside the counters
    int64_t chunk = kNoAllocMaxChunk;
    const size_t qmax = (kNoAllocScratchBytes - kNoAllocCounterBytes) / 2;
    while (chunk > 64 && (size_t)rt::kQueueRegions * rt::sbr_region_capacity(chunk, grid_for(c)) *
                                 sizeof(rt::RayState) > qmax)
        chunk >>= 1;
    const size_t qbytes = (size_t)rt::kQueueRegions * rt::sbr_region_capacity(chunk, grid_for(c)) *
                          sizeof(rt::RayState);
    if (qbytes > qmax) return fail(RT_ERR_CAPACITY, "the ray queues of this device do not fit the fixed scratch");
    unsigned char* base = (unsigned char*)c->scratch;
    FixedQueues fq;
    fq.counters = (uint32_t*)base;
    fq.q[0] = (rt::RayState*)(base + kNoAllocCounterBytes);
    fq.q[1] = (rt::RayState*)(base + kNoAllocCounterBytes + qmax);
    fq.max_chunk = chunk;
    return coverage_impl(c, s, p, tx, rx_ant, g, gain, hits, gain_db, ray_bounces, nullptr, &fq);
}

rt_status rt_coverage_maps(rt_ctx* c, rt_scene* s, const rt_trace_params* p, const rt_device* tx, int32_t ntx,
                           const rt_device* rx_ant, const rt_grid* g, float* gain, uint32_t* hits, float* gain_db) {
    if (!tx || ntx < 1) return fail(RT_ERR_ARG, "need at least one transmitter");
    if (!g || !gain || !hits) return fail(RT_ERR_ARG, "NULL argument");
    const int64_t cells = (int64_t)g->nx * g->ny;
    for (int32_t k = 0; k < ntx; ++k) {
        const rt_status st = coverage_impl(c, s, p, tx + k, rx_ant, g, gain + k * cells, hits + k * cells,
                                           gain_db ? gain_db + k * cells : nullptr, nullptr, nullptr);
        if (st != RT_OK) return st;
    }
    return RT_OK;
}

rt_status rt_coverage_work(rt_ctx* c, rt_scene* s, const rt_trace_params* p, const rt_device* tx,
                           const rt_device* rx_ant, const rt_grid* g, float* gain, uint32_t* hits, uint64_t* work) {
    if (!work) return fail(RT_ERR_ARG, "work is NULL");
    return coverage_impl(c, s, p, tx, rx_ant, g, gain, hits, nullptr, nullptr, work);
}

rt_status rt_profile_enable(rt_ctx* c, int32_t enable) {
    if (!c) return fail(RT_ERR_ARG, "ctx is NULL");
    c->profiling = enable != 0;
    return RT_OK;
}

rt_status rt_profile_read(rt_ctx* c, int32_t n, int64_t* launches, double* ms) {
    if (!c || n < 0 || (n > 0 && (!launches || !ms))) return fail(RT_ERR_ARG, "invalid argument");
    RT_HIP(hipSetDevice(c->device));
    for (int i = 0; i < n; ++i) {
        launches[i] = 0;
        ms[i] = 0.0;
    }
    for (const auto& r : c->recs) {
        RT_HIP(hipEventSynchronize(r.stop));
        float t = 0.0f;
        RT_HIP(hipEventElapsedTime(&t, r.start, r.stop));
        if (r.depth < n) {
            launches[r.depth] += 1;
            ms[r.depth] += t;
        }
    }
    c->recs.clear();
    c->ev_used = 0;
    return RT_OK;
}

rt_status rt_compute_paths(rt_ctx* c, rt_scene* s, const rt_trace_params* p, const rt_device* tx, int32_t ntx,
                           const rt_device* rx, int32_t nrx, float* a, float* T, float* tau, float* aod, float* aoa,
                           int32_t* depth, int32_t* faces, int32_t* num_paths) {
    if (!c || !s || !tx || !rx || !a || !T || !tau || !aod || !aoa || !depth || !faces || !num_paths)
        return fail(RT_ERR_ARG, "NULL argument");
    rt_status st = check_params(p);
    if (st != RT_OK) return st;
    if (ntx < 1 || nrx < 1) return fail(RT_ERR_ARG, "need at least one tx and one rx");
    if (p->max_paths_per_rx < 1 || p->max_paths_per_rx > 256)
        return fail(RT_ERR_ARG, "max_paths_per_rx must be in [1, 256]");
    for (int i = 0; i < ntx; ++i)
        if ((st = check_device(tx + i, "tx", s->host.max_abs)) != RT_OK) return st;
    for (int i = 0; i < nrx; ++i)
        if ((st = check_device(rx + i, "rx", s->host.max_abs)) != RT_OK) return st;
    RT_HIP(hipSetDevice(c->device));
    const bool sphere = p->cand_mode == RT_CAND_SPHERE && p->max_depth > 0;
    if (sphere) {
        if (p->max_depth > rt::kSphereMaxDepth) return fail(RT_ERR_ARG, "reception-sphere mode needs max_depth <= 5");
        if (s->host.num_faces >= rt::kSphereMaxFaces)
            return fail(RT_ERR_ARG, "reception-sphere mode needs fewer than 2^24 faces");
    }
    const int P = p->max_paths_per_rx;
    const int fd = std::max(p->max_depth, 1);
    const int64_t count = traced_count(p);
    // candidate prefix table: power of two >= 2 * (rays * depth), capped at 2^26;
    // in sphere mode it holds only the sequences that reach a receiver
    uint64_t want = std::max<uint64_t>(1024, 2ull * (uint64_t)count * (uint64_t)std::max(p->max_depth, 1));
    if (sphere) want = std::min<uint64_t>(want, 1ull << 22);
    uint64_t cap = 1024;
    while (cap < want && cap < (1ull << 26)) cap <<= 1;
    RT_HIP(ensure(c->table, cap * sizeof(uint64_t)));
    // sphere mode: (receiver, sequence) pair set of 16 entries per path slot of every receiver
    uint64_t pcap = 1024;
    if (sphere)
        while (pcap < 16ull * (uint64_t)nrx * (uint64_t)P && pcap < (1ull << 26)) pcap <<= 1;
    const uint32_t max_cand = (uint32_t)std::min<uint64_t>(sphere ? pcap : cap, 1ull << 24);
    RT_HIP(ensure(c->cands, (size_t)max_cand * sizeof(rt::Cand)));
    RT_HIP(ensure(c->rx, (size_t)nrx * 3 * sizeof(double)));
    RT_HIP(ensure(c->rx_ant, (size_t)nrx * sizeof(rt::Antenna)));
    const size_t per = (size_t)nrx * P;
    const size_t rec_bytes = per * (2 + 8 + 1 + 2 + 2) * sizeof(float) + per * (1 + fd) * sizeof(int32_t) +
                             (size_t)nrx * sizeof(uint32_t) + 3 * sizeof(uint32_t);
    RT_HIP(ensure(c->paths, rec_bytes));
    std::vector<double> rxp(3 * (size_t)nrx);
    std::vector<rt::Antenna> rxa(nrx);
    for (int i = 0; i < nrx; ++i) {
        for (int k = 0; k < 3; ++k) rxp[3 * i + k] = rx[i].pos[k];
        rxa[i] = make_antenna(rx + i);
    }
    // staged on the context's stream: kernels still queued there (a gradient of
    // the previous call) read these buffers
    RT_HIP(hipMemcpyAsync(c->rx.p, rxp.data(), rxp.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    RT_HIP(hipMemcpyAsync(c->rx_ant.p, rxa.data(), rxa.size() * sizeof(rt::Antenna), hipMemcpyHostToDevice,
                          c->stream));
    RT_HIP(hipStreamSynchronize(c->stream));  // host staging vectors go out of scope
    rt::SbrArgs sph{};
    if (sphere) {
        // every accepted pair has a path length below (max_depth + 1) times the
        // diagonal of the box holding the scene, the transmitters and the
        // receivers, so no sphere is wider than r_ins
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        auto grow = [&](double x, double y, double z) {
            const double v[3] = {x, y, z};
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], v[k]);
                hi[k] = std::max(hi[k], v[k]);
            }
        };
        for (const rt::Tri& tr : s->host.tris) {
            grow(tr.v0[0], tr.v0[1], tr.v0[2]);
            grow(tr.v0[0] + tr.e1[0], tr.v0[1] + tr.e1[1], tr.v0[2] + tr.e1[2]);
            grow(tr.v0[0] + tr.e2[0], tr.v0[1] + tr.e2[1], tr.v0[2] + tr.e2[2]);
        }
        for (int i = 0; i < ntx; ++i) grow(tx[i].pos[0], tx[i].pos[1], tx[i].pos[2]);
        double rlo[3] = {1e300, 1e300, 1e300}, rhi[3] = {-1e300, -1e300, -1e300};
        for (int i = 0; i < nrx; ++i) {
            grow(rxp[3 * i], rxp[3 * i + 1], rxp[3 * i + 2]);
            for (int k = 0; k < 3; ++k) {
                rlo[k] = std::min(rlo[k], rxp[3 * i + k]);
                rhi[k] = std::max(rhi[k], rxp[3 * i + k]);
            }
        }
        const double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                      (hi[2] - lo[2]) * (hi[2] - lo[2]));
        sph.sphere_k = (double)p->sphere_kappa * std::sqrt(4.0 * M_PI / (double)count);
        const double r_ins = sph.sphere_k * (p->max_depth + 1) * diag * (1.0 + 1e-9) + 1e-9;
        const double ext = std::max(rhi[0] - rlo[0], rhi[1] - rlo[1]) + 2.0 * r_ins;
        const double cell = std::max(2.0 * r_ins, ext / 1024.0);
        sph.rgx0 = rlo[0] - r_ins;
        sph.rgy0 = rlo[1] - r_ins;
        sph.rgcell = cell;
        sph.rgnx = std::max(1, (int)std::ceil((rhi[0] - rlo[0] + 2.0 * r_ins) / cell));
        sph.rgny = std::max(1, (int)std::ceil((rhi[1] - rlo[1] + 2.0 * r_ins) / cell));
        sph.rz_lo = rlo[2] - r_ins;
        sph.rz_hi = rhi[2] + r_ins;
        // CSR lists: receiver r in every cell that meets the square of half-side r_ins around it
        const int ncell = sph.rgnx * sph.rgny;
        std::vector<int32_t> start(ncell + 1, 0), items;
        auto cell_range = [&](double v, double v0, int n, int& a0, int& a1) {
            a0 = std::min(std::max((int)std::floor((v - r_ins - v0) / cell), 0), n - 1);
            a1 = std::min(std::max((int)std::floor((v + r_ins - v0) / cell), 0), n - 1);
        };
        for (int pass = 0; pass < 2; ++pass) {
            std::vector<int32_t> fill(start.begin(), start.end() - 1);
            for (int i = 0; i < nrx; ++i) {
                int x0, x1, y0, y1;
                cell_range(rxp[3 * i], sph.rgx0, sph.rgnx, x0, x1);
                cell_range(rxp[3 * i + 1], sph.rgy0, sph.rgny, y0, y1);
                for (int iy = y0; iy <= y1; ++iy)
                    for (int ix = x0; ix <= x1; ++ix) {
                        const int cc = iy * sph.rgnx + ix;
                        if (pass == 0) ++start[cc + 1];
                        else items[fill[cc]++] = i;
                    }
            }
            if (pass == 0) {
                for (int k = 0; k < ncell; ++k) start[k + 1] += start[k];
                items.assign(start[ncell], 0);
            }
        }
        RT_HIP(ensure(c->rgrid, (start.size() + items.size()) * sizeof(int32_t)));
        RT_HIP(hipMemcpyAsync(c->rgrid.p, start.data(), start.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                              c->stream));
        if (!items.empty())
            RT_HIP(hipMemcpyAsync((int32_t*)c->rgrid.p + start.size(), items.data(), items.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, c->stream));
        RT_HIP(hipStreamSynchronize(c->stream));
        sph.rx = (const double*)c->rx.p;
        sph.cell_start = (const int32_t*)c->rgrid.p;
        sph.cell_rx = (const int32_t*)c->rgrid.p + start.size();
        RT_HIP(ensure(c->pairs, pcap * sizeof(uint64_t)));
        RT_HIP(ensure(c->pair_rx, (size_t)max_cand * sizeof(int32_t)));
        sph.pairs = (uint64_t*)c->pairs.p;
        sph.pairs_mask = pcap - 1;
    }
    char* base = (char*)c->paths.p;
    rt::PathArgs pa{};
    pa.sc = s->dev;
    pa.freq = p->freq_hz;
    pa.lambda = kC0 / p->freq_hz;
    pa.rx = (const double*)c->rx.p;
    pa.rx_ant = (const rt::Antenna*)c->rx_ant.p;
    pa.nrx = nrx;
    pa.cands = (const rt::Cand*)c->cands.p;
    pa.pair_rx = sphere ? (const int32_t*)c->pair_rx.p : nullptr;
    pa.max_depth = p->max_depth;
    pa.P = P;
    pa.fd = fd;
    pa.a = (float*)base; base += per * 2 * sizeof(float);
    pa.T = (float*)base; base += per * 8 * sizeof(float);
    pa.tau = (float*)base; base += per * sizeof(float);
    pa.aod = (float*)base; base += per * 2 * sizeof(float);
    pa.aoa = (float*)base; base += per * 2 * sizeof(float);
    pa.depth = (int32_t*)base; base += per * sizeof(int32_t);
    pa.faces = (int32_t*)base; base += per * fd * sizeof(int32_t);
    pa.counts = (uint32_t*)base; base += (size_t)nrx * sizeof(uint32_t);
    uint32_t* ncand = (uint32_t*)base;       // [0] candidates, [1] table overflow, [2] pair-set overflow
    pa.ncand = ncand;
    sph.pairs_overflow = ncand + 2;
    rt::MatTable mats = make_mats(s, p->freq_hz);
    int worst = 0;
    std::vector<int32_t> counts_h(nrx);
    for (int t = 0; t < ntx; ++t) {
        RT_HIP(hipMemsetAsync(c->table.p, 0xff, cap * sizeof(uint64_t), c->stream));
        if (sphere) RT_HIP(hipMemsetAsync(c->pairs.p, 0xff, pcap * sizeof(uint64_t), c->stream));
        RT_HIP(hipMemsetAsync(ncand, 0, 3 * sizeof(uint32_t), c->stream));
        RT_HIP(hipMemsetAsync(pa.counts, 0, (size_t)nrx * sizeof(uint32_t), c->stream));
        if (sphere) {
            st = run_sbr(c, s, p, tx + t, nullptr, nullptr, rt::kModeSphere, nullptr, nullptr, nullptr, nullptr,
                         nullptr, (uint64_t*)c->table.p, cap - 1, ncand + 1, nullptr, &sph);
            if (st != RT_OK) return st;
            RT_HIP(rt::launch_extract_pairs((const uint64_t*)c->pairs.p, pcap, (const uint64_t*)c->table.p,
                                            (rt::Cand*)c->cands.p, (int32_t*)c->pair_rx.p, ncand, max_cand,
                                            c->stream));
        } else if (p->max_depth > 0) {
            st = run_sbr(c, s, p, tx + t, nullptr, nullptr, rt::kModeCandidates, nullptr, nullptr, nullptr, nullptr,
                         nullptr, (uint64_t*)c->table.p, cap - 1, ncand + 1);
            if (st != RT_OK) return st;
            RT_HIP(rt::launch_extract_candidates((const uint64_t*)c->table.p, cap, p->max_depth,
                                                 (rt::Cand*)c->cands.p, ncand, max_cand, c->stream));
        }
        uint32_t hc[3] = {0, 0, 0};
        RT_HIP(hipMemcpyAsync(hc, ncand, sizeof(hc), hipMemcpyDeviceToHost, c->stream));
        RT_HIP(hipStreamSynchronize(c->stream));
        if (hc[1]) return fail(RT_ERR_CAPACITY, "candidate table overflow: too many distinct face sequences");
        if (hc[2]) return fail(RT_ERR_CAPACITY, "reception-sphere pair set overflow");
        if (hc[0] > max_cand) return fail(RT_ERR_CAPACITY, "more than 2^24 candidates");
        c->last_candidates = hc[0];
        for (int k = 0; k < 3; ++k) pa.tx[k] = tx[t].pos[k];
        pa.tx_ant = make_antenna(tx + t);
        const int64_t items = sphere ? (int64_t)nrx + (int64_t)hc[0] : (int64_t)nrx * ((int64_t)hc[0] + 1);
        RT_HIP(rt::launch_image_paths(pa, mats, items, c->stream));
        const size_t off = (size_t)t * per;
        RT_HIP(rt::launch_sort_paths(pa, nrx, a + 2 * off, T + 8 * off, tau + off, aod + 2 * off, aoa + 2 * off,
                                     depth + off, faces + (size_t)fd * off, num_paths + (size_t)t * nrx, c->stream));
        RT_HIP(hipMemcpyAsync(counts_h.data(), num_paths + (size_t)t * nrx, (size_t)nrx * sizeof(int32_t),
                              hipMemcpyDeviceToHost, c->stream));
        RT_HIP(hipStreamSynchronize(c->stream));
        for (int i = 0; i < nrx; ++i) worst = std::max(worst, counts_h[i]);
    }
    if (worst > P)
        return fail(RT_ERR_CAPACITY, "a receiver has " + std::to_string(worst) +
                                         " paths; raise max_paths_per_rx to at least that");
    return RT_OK;
}

rt_status rt_paths_power(rt_ctx* c, const float* a, const int32_t* depth, int64_t n, int32_t P, double* power) {
    if (!c || !a || !depth || !power) return fail(RT_ERR_ARG, "NULL argument");
    if (n < 0 || P < 1 || P > 256) return fail(RT_ERR_ARG, "n must be >= 0 and P in [1, 256]");
    RT_HIP(hipSetDevice(c->device));
    RT_HIP(rt::launch_paths_power(a, depth, n, P, power, c->stream));
    return RT_OK;
}

rt_status rt_last_candidate_count(rt_ctx* c, int64_t* count) {
    if (!c || !count) return fail(RT_ERR_ARG, "NULL argument");
    *count = c->last_candidates;
    return RT_OK;
}

rt_status rt_coverage_diffraction(rt_ctx* c, rt_scene* s, double freq_hz, const rt_device* tx,
                                  const rt_device* rx_ant, const rt_grid* g, float* gain) {
    if (!c || !s || !tx || !rx_ant || !g || !gain) return fail(RT_ERR_ARG, "NULL argument");
    if (!(freq_hz > 0) || !std::isfinite(freq_hz)) return fail(RT_ERR_ARG, "freq_hz must be positive");
    rt_status st;
    if ((st = check_device(tx, "tx", s->host.max_abs)) != RT_OK) return st;
    if ((st = check_device(rx_ant, "rx_ant", 0)) != RT_OK) return st;
    if (g->nx < 1 || g->ny < 1 || (int64_t)g->nx * g->ny > (int64_t(1) << 31))
        return fail(RT_ERR_ARG, "grid size must be positive and below 2^31 cells");
    if (!(g->cell > 0) || !std::isfinite(g->cell) || !std::isfinite(g->x0) || !std::isfinite(g->y0) ||
        !std::isfinite(g->z))
        return fail(RT_ERR_ARG, "grid origin, cell size and height must be finite, cell > 0");
    RT_HIP(hipSetDevice(c->device));
    const double txp[3] = {tx->pos[0], tx->pos[1], tx->pos[2]};
    RT_HIP(rt::launch_coverage_diffraction(s->dev, make_mats(s, freq_hz), kC0 / freq_hz, txp, make_antenna(tx),
                                           make_antenna(rx_ant), g->x0, g->y0, g->cell, g->z, g->nx, g->ny, gain,
                                           c->stream));
    return RT_OK;
}

rt_status rt_scene_wedges(const rt_scene* s, int32_t capacity, double* out, int32_t* count) {
    if (!s || !count || (capacity > 0 && !out)) return fail(RT_ERR_ARG, "NULL argument");
    const auto& w = s->host.wedges;
    *count = (int32_t)w.size();
    for (int32_t i = 0; i < capacity && i < (int32_t)w.size(); ++i) {
        double* o = out + 16 * (size_t)i;
        for (int k = 0; k < 3; ++k) {
            o[k] = w[i].a[k];
            o[3 + k] = w[i].e[k];
            o[6 + k] = w[i].t0[k];
            o[9 + k] = w[i].n0[k];
        }
        o[12] = w[i].len;
        o[13] = w[i].n;
        o[14] = w[i].face0;
        o[15] = w[i].facen;
    }
    return RT_OK;
}

rt_status rt_compute_diffraction(rt_ctx* c, rt_scene* s, double freq_hz, const rt_device* tx, int32_t ntx,
                                 const rt_device* rx, int32_t nrx, int32_t P, float* a, float* T, float* tau,
                                 float* aod, float* aoa, int32_t* wedge, int32_t* num_paths) {
    if (!c || !s || !tx || !rx || !a || !T || !tau || !aod || !aoa || !wedge || !num_paths)
        return fail(RT_ERR_ARG, "NULL argument");
    if (!(freq_hz > 0) || !std::isfinite(freq_hz)) return fail(RT_ERR_ARG, "freq_hz must be positive");
    if (ntx < 1 || nrx < 1) return fail(RT_ERR_ARG, "need at least one tx and one rx");
    if (P < 1 || P > 256) return fail(RT_ERR_ARG, "P must be in [1, 256]");
    rt_status st;
    for (int i = 0; i < ntx; ++i)
        if ((st = check_device(tx + i, "tx", s->host.max_abs)) != RT_OK) return st;
    for (int i = 0; i < nrx; ++i)
        if ((st = check_device(rx + i, "rx", s->host.max_abs)) != RT_OK) return st;
    RT_HIP(hipSetDevice(c->device));
    const size_t per = (size_t)nrx * P;
    // unsorted records (fd = 1: the wedge id in the faces slot), the sorted
    // depths the sort writes, and the per-receiver counts
    const size_t rec_bytes = per * (2 + 8 + 1 + 2 + 2) * sizeof(float) + per * 3 * sizeof(int32_t) +
                             (size_t)nrx * sizeof(uint32_t);
    RT_HIP(ensure(c->paths, rec_bytes));
    RT_HIP(ensure(c->rx, (size_t)nrx * 3 * sizeof(double)));
    RT_HIP(ensure(c->rx_ant, (size_t)nrx * sizeof(rt::Antenna)));
    std::vector<double> rxp(3 * (size_t)nrx);
    std::vector<rt::Antenna> rxa(nrx);
    for (int i = 0; i < nrx; ++i) {
        for (int k = 0; k < 3; ++k) rxp[3 * i + k] = rx[i].pos[k];
        rxa[i] = make_antenna(rx + i);
    }
    RT_HIP(hipMemcpyAsync(c->rx.p, rxp.data(), rxp.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    RT_HIP(hipMemcpyAsync(c->rx_ant.p, rxa.data(), rxa.size() * sizeof(rt::Antenna), hipMemcpyHostToDevice,
                          c->stream));
    RT_HIP(hipStreamSynchronize(c->stream));  // host staging vectors go out of scope
    char* base = (char*)c->paths.p;
    rt::PathArgs pa{};
    pa.sc = s->dev;
    pa.freq = freq_hz;
    pa.lambda = kC0 / freq_hz;
    pa.rx = (const double*)c->rx.p;
    pa.rx_ant = (const rt::Antenna*)c->rx_ant.p;
    pa.nrx = nrx;
    pa.P = P;
    pa.fd = 1;
    pa.a = (float*)base; base += per * 2 * sizeof(float);
    pa.T = (float*)base; base += per * 8 * sizeof(float);
    pa.tau = (float*)base; base += per * sizeof(float);
    pa.aod = (float*)base; base += per * 2 * sizeof(float);
    pa.aoa = (float*)base; base += per * 2 * sizeof(float);
    pa.depth = (int32_t*)base; base += per * sizeof(int32_t);
    pa.faces = (int32_t*)base; base += per * sizeof(int32_t);
    int32_t* depth_sorted = (int32_t*)base; base += per * sizeof(int32_t);
    pa.counts = (uint32_t*)base;
    rt::MatTable mats = make_mats(s, freq_hz);
    int worst = 0;
    std::vector<int32_t> counts_h(nrx);
    for (int t = 0; t < ntx; ++t) {
        for (int i = 0; i < 3; ++i) pa.tx[i] = tx[t].pos[i];
        pa.tx_ant = make_antenna(tx + t);
        RT_HIP(hipMemsetAsync(pa.counts, 0, (size_t)nrx * sizeof(uint32_t), c->stream));
        RT_HIP(rt::launch_diffraction_paths(pa, mats, c->stream));
        const size_t off = (size_t)t * per;
        RT_HIP(rt::launch_sort_paths(pa, nrx, a + 2 * off, T + 8 * off, tau + off, aod + 2 * off, aoa + 2 * off,
                                     depth_sorted, wedge + off, num_paths + (size_t)t * nrx, c->stream));
        RT_HIP(hipMemcpyAsync(counts_h.data(), num_paths + (size_t)t * nrx, (size_t)nrx * sizeof(int32_t),
                              hipMemcpyDeviceToHost, c->stream));
        RT_HIP(hipStreamSynchronize(c->stream));
        for (int i = 0; i < nrx; ++i) worst = std::max(worst, counts_h[i]);
    }
    if (worst > P)
        return fail(RT_ERR_CAPACITY, "a receiver has " + std::to_string(worst) +
                                         " diffracted paths; raise P to at least that");
    return RT_OK;
}

rt_status rt_compute_scattering(rt_ctx* c, rt_scene* s, const rt_trace_params* p, const rt_device* tx, int32_t ntx,
                                const rt_device* rx, int32_t nrx, int64_t P, float* a, float* T, float* tau,
                                float* aod, float* aoa, int32_t* depth, int64_t* ray, int32_t* faces,
                                int64_t* num_paths) {
    if (!c || !s || !tx || !rx || !a || !T || !tau || !aod || !aoa || !depth || !ray || !faces || !num_paths)
        return fail(RT_ERR_ARG, "NULL argument");
    rt_status st = check_params(p);
    if (st != RT_OK) return st;
    if (ntx < 1 || nrx < 1) return fail(RT_ERR_ARG, "need at least one tx and one rx");
    if (P < 1 || P > (int64_t(1) << 40)) return fail(RT_ERR_ARG, "P must be in [1, 2^40]");
    for (int i = 0; i < ntx; ++i)
        if ((st = check_device(tx + i, "tx", s->host.max_abs)) != RT_OK) return st;
    for (int i = 0; i < nrx; ++i)
        if ((st = check_device(rx + i, "rx", s->host.max_abs)) != RT_OK) return st;
    RT_HIP(hipSetDevice(c->device));
    const int D = p->max_depth;
    const int fd = std::max(D, 1);
    const int64_t count = traced_count(p);
    // chunk of rays: records, masks and prefixes within about 1 GiB
    const int64_t per_ray = (int64_t)std::max(D, 1) * (int64_t)(sizeof(rt::ScatPoint) + (nrx * 12 + 63) / 64);
    int64_t chunk = std::min<int64_t>(int64_t(1) << 20, std::max<int64_t>(64, (int64_t(1) << 30) / per_ray));
    chunk = std::min<int64_t>(chunk, count);
    const int64_t nrec_pad = (chunk * std::max(D, 1) + 63) / 64 * 64;
    const int64_t nwords = nrec_pad / 64;
    const size_t pts_bytes = (size_t)chunk * std::max(D, 1) * sizeof(rt::ScatPoint);
    const size_t mask_bytes = (size_t)nrx * nwords * sizeof(uint64_t);
    const size_t pre_bytes = ((size_t)nrx * nwords * sizeof(uint32_t) + 255) / 256 * 256;
    const size_t cnt_bytes = (size_t)nrx * 2 * sizeof(int64_t);
    RT_HIP(ensure(c->scat, pts_bytes + mask_bytes + pre_bytes + cnt_bytes));
    RT_HIP(ensure(c->rx, (size_t)nrx * 3 * sizeof(double)));
    RT_HIP(ensure(c->rx_ant, (size_t)nrx * sizeof(rt::Antenna)));
    std::vector<double> rxp(3 * (size_t)nrx);
    std::vector<rt::Antenna> rxa(nrx);
    for (int i = 0; i < nrx; ++i) {
        for (int k = 0; k < 3; ++k) rxp[3 * i + k] = rx[i].pos[k];
        rxa[i] = make_antenna(rx + i);
    }
    RT_HIP(hipMemcpyAsync(c->rx.p, rxp.data(), rxp.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    RT_HIP(hipMemcpyAsync(c->rx_ant.p, rxa.data(), rxa.size() * sizeof(rt::Antenna), hipMemcpyHostToDevice,
                          c->stream));
    RT_HIP(hipStreamSynchronize(c->stream));  // host staging vectors go out of scope
    char* buf = (char*)c->scat.p;
    rt::ScatArgs sa{};
    sa.sc = s->dev;
    sa.num_rays = p->num_rays;
    sa.begin = p->ray_begin;
    sa.stride = p->ray_stride;
    sa.max_depth = D;
    sa.nrx = nrx;
    sa.tmin = p->t_min;
    sa.lambda = kC0 / p->freq_hz;
    sa.rx = (const double*)c->rx.p;
    sa.rx_ant = (const rt::Antenna*)c->rx_ant.p;
    sa.points = (rt::ScatPoint*)buf; buf += pts_bytes;
    sa.nrec_pad = nrec_pad;
    sa.masks = (uint64_t*)buf; buf += mask_bytes;
    sa.prefix = (uint32_t*)buf; buf += pre_bytes;
    sa.chunk_total = (int64_t*)buf;
    sa.P = P;
    sa.fd = fd;
    rt::MatTable mats = make_mats(s, p->freq_hz);
    int64_t worst = 0;
    std::vector<int64_t> counts_h(nrx);
    for (int t = 0; t < ntx; ++t) {
        for (int i = 0; i < 3; ++i) sa.tx[i] = tx[t].pos[i];
        sa.tx_ant = make_antenna(tx + t);
        const size_t off = (size_t)t * nrx * P;
        sa.a = a + 2 * off;
        sa.T = T + 8 * off;
        sa.tau = tau + off;
        sa.aod = aod + 2 * off;
        sa.aoa = aoa + 2 * off;
        sa.depth = depth + off;
        sa.ray = ray + off;
        sa.faces = faces + off * fd;
        sa.base = num_paths + (size_t)t * nrx;
        RT_HIP(rt::launch_fill_u32(sa.base, 0u, (size_t)nrx * 2, c->stream));
        for (int64_t pos0 = 0; pos0 < count; pos0 += chunk) {
            sa.pos0 = pos0;
            sa.n = std::min<int64_t>(chunk, count - pos0);
            RT_HIP(rt::launch_scatter_chunk(sa, mats, c->stream));
        }
        RT_HIP(rt::launch_scatter_tail(sa, c->stream));
        RT_HIP(hipMemcpyAsync(counts_h.data(), sa.base, (size_t)nrx * sizeof(int64_t), hipMemcpyDeviceToHost,
                              c->stream));
        RT_HIP(hipStreamSynchronize(c->stream));
        for (int i = 0; i < nrx; ++i) worst = std::max(worst, counts_h[i]);
    }
    if (worst > P)
        return fail(RT_ERR_CAPACITY, "a receiver has " + std::to_string(worst) +
                                         " scattered paths; raise P to at least that");
    return RT_OK;
}

// Gradient of received powers (dL_dP) or of any function of the path
// coefficients given their complex adjoints (coef_adj); exactly one is set.
static rt_status paths_grad_impl(rt_ctx* c, rt_scene* s, const rt_trace_params* p, const rt_device* tx,
                                 const rt_device* rx, int32_t nrx, int32_t P, const int32_t* depth,
                                 const int32_t* faces, const double* dL_dP, const double* coef_adj, double* grad) {
    if (!c || !s || !rx || !depth || !faces || !(dL_dP || coef_adj) || !grad) return fail(RT_ERR_ARG, "NULL argument");
    rt_status st = check_params(p);
    if (st != RT_OK) return st;
    if ((st = check_device(tx, "tx", s->host.max_abs)) != RT_OK) return st;
    if (nrx < 1 || P < 1 || P > 256) return fail(RT_ERR_ARG, "nrx must be >= 1 and P in [1, 256]");
    for (int i = 0; i < nrx; ++i)
        if ((st = check_device(rx + i, "rx", s->host.max_abs)) != RT_OK) return st;
    RT_HIP(hipSetDevice(c->device));
    RT_HIP(ensure(c->rx, (size_t)nrx * 3 * sizeof(double)));
    RT_HIP(ensure(c->rx_ant, (size_t)nrx * sizeof(rt::Antenna)));
    std::vector<double> rxp(3 * (size_t)nrx);
    std::vector<rt::Antenna> rxa(nrx);
    for (int i = 0; i < nrx; ++i) {
        for (int k = 0; k < 3; ++k) rxp[3 * i + k] = rx[i].pos[k];
        rxa[i] = make_antenna(rx + i);
    }
    RT_HIP(hipMemcpyAsync(c->rx.p, rxp.data(), rxp.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    RT_HIP(hipMemcpyAsync(c->rx_ant.p, rxa.data(), rxa.size() * sizeof(rt::Antenna), hipMemcpyHostToDevice,
                          c->stream));
    RT_HIP(hipStreamSynchronize(c->stream));  // host staging vectors go out of scope
    const int nm = (int)s->mats.size();
    RT_HIP(hipMemsetAsync(grad, 0, (size_t)(2 * nm + 5) * sizeof(double), c->stream));
    rt::GradArgs g{};
    g.sc = s->dev;
    g.freq = p->freq_hz;
    g.lambda = kC0 / p->freq_hz;
    for (int k = 0; k < 3; ++k) g.tx[k] = tx->pos[k];
    g.yaw = tx->yaw;
    g.pitch = tx->pitch;
    g.roll = tx->roll;
    g.tx_pattern = tx->pattern;
    g.tx_pol = tx->pol;
    g.rx = (const double*)c->rx.p;
    g.rx_ant = (const rt::Antenna*)c->rx_ant.p;
    g.nrx = nrx;
    g.P = P;
    g.fd = std::max(p->max_depth, 1);
    g.depth = depth;
    g.faces = faces;
    g.dL_dP = dL_dP;
    g.coef_adj = coef_adj;
    g.grad = grad;
    g.nm = nm;
    RT_HIP(rt::launch_power_grad(g, make_mats(s, p->freq_hz), c->stream));
    return RT_OK;
}

rt_status rt_paths_power_grad(rt_ctx* c, rt_scene* s, const rt_trace_params* p, const rt_device* tx,
                              const rt_device* rx, int32_t nrx, int32_t P, const int32_t* depth,
                              const int32_t* faces, const double* dL_dP, double* grad) {
    if (!dL_dP) return fail(RT_ERR_ARG, "NULL argument");
    return paths_grad_impl(c, s, p, tx, rx, nrx, P, depth, faces, dL_dP, nullptr, grad);
}

rt_status rt_coverage_grad(rt_ctx* c, rt_scene* s, const rt_trace_params* p, const rt_device* tx,
                           const rt_device* rx_ant, const rt_grid* g, const uint8_t* region, const int32_t* hit_tri,
                           const double* hit_t, double* out) {
    if (!c || !s || !g || !hit_tri || !hit_t || !out) return fail(RT_ERR_ARG, "NULL argument");
    rt_status st = check_params(p);
    if (st != RT_OK) return st;
    if ((st = check_device(tx, "tx", s->host.max_abs)) != RT_OK) return st;
    if ((st = check_device(rx_ant, "rx_ant", 0)) != RT_OK) return st;
    if (g->nx < 1 || g->ny < 1 || (int64_t)g->nx * g->ny > (int64_t(1) << 31))
        return fail(RT_ERR_ARG, "grid size must be positive and below 2^31 cells");
    if (!(g->cell > 0) || !std::isfinite(g->cell) || !std::isfinite(g->x0) || !std::isfinite(g->y0) ||
        !std::isfinite(g->z))
        return fail(RT_ERR_ARG, "grid origin, cell size and height must be finite, cell > 0");
    const int nm = (int)s->mats.size();
    if (nm > rt::kCovMaxMat) return fail(RT_ERR_ARG, "coverage gradient supports at most 4 materials");
    RT_HIP(hipSetDevice(c->device));
    RT_HIP(hipMemsetAsync(out, 0, (size_t)(2 * nm + 3) * sizeof(double), c->stream));
    rt::CovGradArgs a{};
    a.sc = s->dev;
    a.num_rays = p->num_rays;
    a.begin = p->ray_begin;
    a.stride = p->ray_stride;
    a.count = traced_count(p);
    a.max_depth = p->max_depth;
    a.nm = nm;
    for (int k = 0; k < 3; ++k) a.tx[k] = tx->pos[k];
    a.yaw = tx->yaw;
    a.pitch = tx->pitch;
    a.roll = tx->roll;
    a.tx_pattern = tx->pattern;
    a.tx_pol = tx->pol;
    a.gnx = g->nx;
    a.gny = g->ny;
    a.rx_ant = make_antenna(rx_ant);
    a.gx0 = g->x0;
    a.gy0 = g->y0;
    a.gcell = g->cell;
    a.gz = g->z;
    const double lam = kC0 / p->freq_hz;
    a.wscale = (lam / (4.0 * M_PI)) * (lam / (4.0 * M_PI)) * (4.0 * M_PI / (double)p->num_rays) / (g->cell * g->cell);
    a.omega = 2.0 * M_PI * p->freq_hz;
    a.scat_seed = s->scat_seed;
    a.region = region;
    a.hit_tri = hit_tri;
    a.hit_t = hit_t;
    a.out = out;
    RT_HIP(rt::launch_coverage_grad(a, make_mats(s, p->freq_hz), grid_for(c), c->stream));
    return RT_OK;
}

}  // extern "C"

namespace {
// Validates the channel-response arguments and stages the small host arrays
// (element offsets, velocities) in the context's device buffer.
rt_status cfr_setup(rt_ctx* c, int32_t ntx, int32_t nrx, int32_t P, const float* a, const float* tau,
                    const float* aod, const float* aoa, const int32_t* depth, double freq_hz, int32_t K,
                    double spacing_hz, int32_t nt_el, const double* tx_el, int32_t nr_el, const double* rx_el,
                    const double* v_tx, const double* v_rx, int32_t T, double fs, const void* out_a,
                    const void* out_b, rt::CfrArgs& cf) {
    if (!c || !a || !tau || !aod || !aoa || !depth) return fail(RT_ERR_ARG, "NULL argument");
    if (ntx < 1 || nrx < 1 || P < 1) return fail(RT_ERR_ARG, "ntx, nrx and P must be >= 1");
    if (!(freq_hz > 0) || !std::isfinite(freq_hz)) return fail(RT_ERR_ARG, "frequency must be positive");
    if (K < 1 || !(spacing_hz >= 0) || !std::isfinite(spacing_hz))
        return fail(RT_ERR_ARG, "need K >= 1 subcarriers and a finite spacing >= 0");
    if (nt_el < 1 || nr_el < 1 || (nt_el > 1 && !tx_el) || (nr_el > 1 && !rx_el))
        return fail(RT_ERR_ARG, "arrays need >= 1 element and offsets for more than one");
    if (T < 1 || (T > 1 && !(fs > 0 && std::isfinite(fs))))
        return fail(RT_ERR_ARG, "need T >= 1 time steps and a positive sampling frequency for T > 1");
    std::vector<double> h;
    auto put = [&](const double* src, int64_t n) {
        for (int64_t i = 0; i < n; ++i) {
            const double v = src ? src[i] : 0.0;
            h.push_back(v);
        }
    };
    put(tx_el, 3 * (int64_t)nt_el);
    put(rx_el, 3 * (int64_t)nr_el);
    put(v_tx, 3 * (int64_t)ntx);
    put(v_rx, 3 * (int64_t)nrx);
    for (double v : h)
        if (!std::isfinite(v)) return fail(RT_ERR_ARG, "element offsets and velocities must be finite");
    if (!out_a || !out_b) return fail(RT_ERR_ARG, "NULL argument");
    RT_HIP(hipSetDevice(c->device));
    RT_HIP(ensure(c->chan, h.size() * sizeof(double)));
    RT_HIP(hipMemcpyAsync(c->chan.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    RT_HIP(hipStreamSynchronize(c->stream));  // the staging vector goes out of scope
    const double* d = (const double*)c->chan.p;
    cf = rt::CfrArgs{};
    cf.npairs = (int64_t)ntx * nrx;
    cf.nrx = nrx;
    cf.P = P;
    cf.a = a;
    cf.tau = tau;
    cf.aod = aod;
    cf.aoa = aoa;
    cf.depth = depth;
    cf.freq = freq_hz;
    cf.lambda = kC0 / freq_hz;
    cf.spacing = spacing_hz;
    cf.fs = T > 1 ? fs : 1.0;
    cf.K = K;
    cf.T = T;
    cf.nt_el = nt_el;
    cf.nr_el = nr_el;
    cf.tx_el = d;
    cf.rx_el = d + 3 * nt_el;
    cf.v_tx = d + 3 * (nt_el + nr_el);
    cf.v_rx = d + 3 * (nt_el + nr_el + ntx);
    cf.total = cf.npairs * T * nr_el * nt_el * K;
    return RT_OK;
}
}  // namespace

extern "C" {

rt_status rt_paths_cfr(rt_ctx* c, int32_t ntx, int32_t nrx, int32_t P, const float* a, const float* tau,
                       const float* aod, const float* aoa, const int32_t* depth, double freq_hz, int32_t K,
                       double spacing_hz, int32_t nt_el, const double* tx_el, int32_t nr_el, const double* rx_el,
                       const double* v_tx, const double* v_rx, int32_t T, double fs, float* H) {
    rt::CfrArgs cf;
    rt_status st = cfr_setup(c, ntx, nrx, P, a, tau, aod, aoa, depth, freq_hz, K, spacing_hz, nt_el, tx_el, nr_el,
                             rx_el, v_tx, v_rx, T, fs, H, H, cf);
    if (st != RT_OK) return st;
    cf.H = H;
    RT_HIP(rt::launch_cfr(cf, c->stream));
    return RT_OK;
}

rt_status rt_paths_cfr_adjoint(rt_ctx* c, int32_t ntx, int32_t nrx, int32_t P, const float* a, const float* tau,
                               const float* aod, const float* aoa, const int32_t* depth, double freq_hz, int32_t K,
                               double spacing_hz, int32_t nt_el, const double* tx_el, int32_t nr_el,
                               const double* rx_el, const double* v_tx, const double* v_rx, int32_t T, double fs,
                               const float* G, double* g) {
    rt::CfrArgs cf;
    rt_status st = cfr_setup(c, ntx, nrx, P, a, tau, aod, aoa, depth, freq_hz, K, spacing_hz, nt_el, tx_el, nr_el,
                             rx_el, v_tx, v_rx, T, fs, G, g, cf);
    if (st != RT_OK) return st;
    RT_HIP(rt::launch_cfr_adjoint(cf, G, g, c->stream));
    return RT_OK;
}

rt_status rt_paths_coef_grad(rt_ctx* c, rt_scene* s, const rt_trace_params* p, const rt_device* tx,
                             const rt_device* rx, int32_t nrx, int32_t P, const int32_t* depth, const int32_t* faces,
                             const double* coef_adj, double* grad) {
    if (!coef_adj) return fail(RT_ERR_ARG, "NULL argument");
    return paths_grad_impl(c, s, p, tx, rx, nrx, P, depth, faces, nullptr, coef_adj, grad);
}

}  // extern "C"
