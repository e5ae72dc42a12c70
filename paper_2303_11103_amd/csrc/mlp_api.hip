// C ABI of the MLP surrogate (declared in include/rt.h): handle with fp32
// master weights, Adam state, bf16 weight copies and per-batch scratch; the
// launch sequences of forward, gradient, training step, batch sampling and
// map prediction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mlp_kernels.h"
#include "rt.h"

rt_status rt_internal_fail(rt_status code, const char* msg);
hipStream_t rt_internal_stream(rt_ctx* c);
int rt_internal_device(rt_ctx* c);
rt_ctx* rt_internal_scene_ctx(const rt_scene* s);

namespace {

#define MLP_HIP(call)                                                                                 \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            return rt_internal_fail(e_ == hipErrorOutOfMemory ? RT_ERR_OOM : RT_ERR_DEVICE,           \
                                    (std::string(#call) + ": " + hipGetErrorString(e_)).c_str());     \
    } while (0)

constexpr int kHidden = 256;
constexpr int kSplits = 64;

rt::MlpLayout make_layout() {
    rt::MlpLayout L{};
    int64_t off = 0, bf = 0;
    const int fan[5] = {2 * rt::kFreq, kHidden, kHidden, kHidden, kHidden};
    const int outs[5] = {kHidden, kHidden, kHidden, kHidden, 1};
    for (int l = 0; l < 5; ++l) {
        L.fan_in[l] = fan[l];
        L.w_off[l] = off;
        L.w_size[l] = (int64_t)fan[l] * outs[l];
        off += L.w_size[l];
        L.b_off[l] = off;
        off += outs[l];
        if (l < 4) {
            L.bf_off[l] = bf;
            bf += L.w_size[l];
        }
    }
    L.total = off;
    return L;
}

}  // namespace

struct rt_mlp {
    rt_ctx* ctx = nullptr;
    rt_mlp_config cfg{};
    rt::MlpLayout lay{};
    rt::MlpNorm norm{};
    int64_t nbf = 0;
    float *params = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr, *ff = nullptr;
    __bf16 *wbf = nullptr, *wtbf = nullptr;
    // batch scratch (rows = cfg.batch)
    __bf16 *feats = nullptr, *Z[4] = {}, *H[4] = {}, *dZa = nullptr, *dZb = nullptr, *T1 = nullptr, *T2 = nullptr;
    float *part = nullptr, *scal = nullptr, *pred = nullptr, *vin = nullptr;  // scal: [0] mask sum, [1] loss
    _Float16* wfrag = nullptr;  // map inference: fragment-major f16 weights
    int num_cu = 256;
    int64_t step = 0;
    std::vector<void*> allocs;
    // ray-tracer fallback scratch (grown on demand, freed on destroy)
    float* fb_tx = nullptr;
    size_t fb_tx_n = 0;
    float* fb_gain = nullptr;
    uint32_t* fb_hits = nullptr;
    size_t fb_cells = 0;
    unsigned long long* fb_count = nullptr;
};

namespace {

template <typename T>
hipError_t alloc(rt_mlp* h, T** p, size_t n) {
    hipError_t e = hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T));
    if (e == hipSuccess) h->allocs.push_back(*p);
    return e;
}

rt_status check_rows(const rt_mlp* h, int64_t n) {
    if (n < 128 || n > h->cfg.batch || n % 128)
        return rt_internal_fail(RT_ERR_ARG, "row count must be a multiple of 128 in [128, batch]");
    return RT_OK;
}

// Forward pass over n rows whose raw inputs are in v (device, [n][5]).
rt_status forward(rt_mlp* h, const float* v, int64_t n, hipStream_t s) {
    MLP_HIP(rt::launch_features(v, n, h->ff, h->norm, h->feats, s));
    const __bf16* in = h->feats;
    for (int l = 0; l < 4; ++l) {
        rt::GemmArgs g{};
        g.A = in;
        g.lda = h->lay.fan_in[l];
        g.B = h->wbf + h->lay.bf_off[l];
        g.ldb = h->lay.fan_in[l];
        g.M = (int)n;
        g.N = kHidden;
        g.K = h->lay.fan_in[l];
        g.ksplit = g.K;
        g.epi = rt::kEpiBiasGelu;
        g.bias = h->params + h->lay.b_off[l];
        g.outZ = h->Z[l];
        g.outH = h->H[l];
        MLP_HIP(rt::launch_gemm_nt(g, 1, s));
        in = h->H[l];
    }
    return RT_OK;
}

// Gradient of the masked MSE over n rows into h->grad (zeroed first); loss
// into h->scal[1].
rt_status gradient(rt_mlp* h, const float* v, const float* t, const float* m, int64_t n, hipStream_t s) {
    rt_status st = forward(h, v, n, s);
    if (st != RT_OK) return st;
    const rt::MlpLayout& L = h->lay;
    MLP_HIP(hipMemsetAsync(h->grad, 0, (size_t)L.total * sizeof(float), s));
    MLP_HIP(hipMemsetAsync(h->scal, 0, 2 * sizeof(float), s));
    MLP_HIP(rt::launch_mask_sum(m, n, h->scal, s));
    MLP_HIP(rt::launch_head(h->H[3], h->Z[3], h->params + L.w_off[4], h->params + L.b_off[4], v, h->norm, t, m, n,
                            h->scal, h->pred, h->scal + 1, h->dZa, h->grad + L.w_off[4], h->grad + L.b_off[4], s));
    __bf16* dz = h->dZa;
    __bf16* dz_next = h->dZb;
    for (int l = 3; l >= 0; --l) {
        const int K = L.fan_in[l];
        // dW_l = dZ_l^T H_{l-1}: both operands transposed so that rows are the reduction axis
        MLP_HIP(rt::launch_transpose(dz, n, kHidden, h->T1, s));
        MLP_HIP(rt::launch_rowsum(h->T1, kHidden, n, h->grad + L.b_off[l], s));  // db_l = column sums of dZ_l
        const __bf16* hp = l ? h->H[l - 1] : h->feats;
        MLP_HIP(rt::launch_transpose(hp, n, K, h->T2, s));
        int S = kSplits;
        while (S > 1 && (n / S) % 32) S >>= 1;
        rt::GemmArgs g{};
        g.A = h->T1;
        g.lda = (int)n;
        g.B = h->T2;
        g.ldb = (int)n;
        g.M = kHidden;
        g.N = K;
        g.K = (int)n;
        g.ksplit = (int)(n / S);
        g.epi = rt::kEpiStoreF32;
        g.outF = h->part;
        MLP_HIP(rt::launch_gemm_nt(g, S, s));
        MLP_HIP(rt::launch_reduce_splits(h->part, S, (int64_t)kHidden * K, h->grad + L.w_off[l], s));
        if (l > 0) {
            rt::GemmArgs d{};
            d.A = dz;
            d.lda = kHidden;
            d.B = h->wtbf + L.bf_off[l];
            d.ldb = kHidden;
            d.M = (int)n;
            d.N = K;
            d.K = kHidden;
            d.ksplit = kHidden;
            d.epi = rt::kEpiGeluGrad;
            d.Zprev = h->Z[l - 1];
            d.outZ = dz_next;
            MLP_HIP(rt::launch_gemm_nt(d, 1, s));
            std::swap(dz, dz_next);
        }
    }
    return RT_OK;
}

}  // namespace

extern "C" {

rt_status rt_mlp_param_count(int64_t* n) {
    if (!n) return rt_internal_fail(RT_ERR_ARG, "NULL argument");
    *n = make_layout().total;
    return RT_OK;
}

rt_status rt_mlp_create(rt_ctx* c, const rt_mlp_config* cfg, rt_mlp** out) {
    if (!c || !cfg || !out) return rt_internal_fail(RT_ERR_ARG, "NULL argument");
    if (cfg->batch < 128 || cfg->batch % 1024 || cfg->batch > (1 << 22))
        return rt_internal_fail(RT_ERR_ARG, "batch must be a multiple of 1024 in [1024, 2^22]");
    for (int i = 0; i < 5; ++i)
        if (!(cfg->in_half[i] > 0) || !std::isfinite(cfg->in_center[i]))
            return rt_internal_fail(RT_ERR_ARG, "input normalisation needs finite centres and positive half-ranges");
    if (!(cfg->ff_scale > 0)) return rt_internal_fail(RT_ERR_ARG, "ff_scale must be positive");
    if (!(cfg->ff_scale_cell >= 0) || !std::isfinite(cfg->ff_scale_cell))
        return rt_internal_fail(RT_ERR_ARG, "ff_scale_cell must be >= 0 (0 = ff_scale)");
    if (!(cfg->prior_freq_hz >= 0) || !std::isfinite(cfg->prior_freq_hz) || !std::isfinite(cfg->prior_rx_z))
        return rt_internal_fail(RT_ERR_ARG, "prior_freq_hz must be >= 0 and prior_rx_z finite");
    if (cfg->ff_rows_tx < 0 || cfg->ff_rows_rel < 0 || cfg->ff_rows_tx + cfg->ff_rows_rel > rt::kFreq)
        return rt_internal_fail(RT_ERR_ARG, "ff_rows_tx, ff_rows_rel must be >= 0 with a sum <= 64");
    if (cfg->ff_rows_rel > 0 && (!(cfg->ff_scale_rel > 0) || !std::isfinite(cfg->ff_scale_rel)))
        return rt_internal_fail(RT_ERR_ARG, "ff_scale_rel must be positive");
    MLP_HIP(hipSetDevice(rt_internal_device(c)));
    rt_mlp* h = new rt_mlp();
    h->ctx = c;
    h->cfg = *cfg;
    h->lay = make_layout();
    for (int i = 0; i < 5; ++i) {
        h->norm.center[i] = cfg->in_center[i];
        h->norm.inv_half[i] = 1.0f / cfg->in_half[i];
    }
    h->norm.prior_on = cfg->prior_freq_hz > 0 ? 1 : 0;
    h->norm.prior_rx_z = cfg->prior_rx_z;
    h->norm.prior_db = h->norm.prior_on ? (float)(20.0 * std::log10(299792458.0 / (4.0 * M_PI * cfg->prior_freq_hz)))
                                        : 0.0f;
    const int64_t P = h->lay.total, B = cfg->batch;
    h->nbf = h->lay.bf_off[3] + h->lay.w_size[3];
    hipError_t e = hipSuccess;
    auto A = [&](auto** p, size_t n) {
        if (e == hipSuccess) e = alloc(h, p, n);
    };
    A(&h->params, P);
    A(&h->grad, P);
    A(&h->m1, P);
    A(&h->m2, P);
    A(&h->ff, rt::kFreq * 5);
    A(&h->wbf, h->nbf);
    A(&h->wtbf, h->nbf);
    A(&h->feats, B * 2 * rt::kFreq);
    for (int l = 0; l < 4; ++l) {
        A(&h->Z[l], B * kHidden);
        A(&h->H[l], B * kHidden);
    }
    A(&h->dZa, B * kHidden);
    A(&h->dZb, B * kHidden);
    A(&h->T1, B * kHidden);
    A(&h->T2, B * kHidden);
    A(&h->part, (size_t)kSplits * kHidden * kHidden);
    A(&h->scal, 4);
    A(&h->pred, B);
    A(&h->vin, B * 5);
    A(&h->wfrag, (size_t)rt::v2_weights_halves());
    {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, rt_internal_device(c)) == hipSuccess &&
            cu > 0)
            h->num_cu = cu;
    }
    hipStream_t s = rt_internal_stream(c);
    if (e == hipSuccess) e = hipMemsetAsync(h->m1, 0, P * sizeof(float), s);
    if (e == hipSuccess) e = hipMemsetAsync(h->m2, 0, P * sizeof(float), s);
    rt::MlpFourier fs{cfg->ff_scale, cfg->ff_scale_cell > 0 ? cfg->ff_scale_cell : cfg->ff_scale, cfg->ff_scale_rel,
                      cfg->ff_rows_tx, cfg->ff_rows_rel};
    if (e == hipSuccess) e = rt::launch_mlp_init(h->params, h->ff, cfg->seed, fs, h->lay, s);
    if (e == hipSuccess) e = rt::launch_refresh_bf16(h->params, h->lay, h->wbf, h->wtbf, s);
    if (e != hipSuccess) {
        rt_mlp_destroy(h);
        return rt_internal_fail(e == hipErrorOutOfMemory ? RT_ERR_OOM : RT_ERR_DEVICE, hipGetErrorString(e));
    }
    *out = h;
    return RT_OK;
}

rt_status rt_mlp_destroy(rt_mlp* h) {
    if (!h) return RT_OK;
    (void)hipSetDevice(rt_internal_device(h->ctx));
    (void)hipStreamSynchronize(rt_internal_stream(h->ctx));
    for (void* p : h->allocs) (void)hipFree(p);
    for (void* p : {(void*)h->fb_tx, (void*)h->fb_gain, (void*)h->fb_hits, (void*)h->fb_count})
        if (p) (void)hipFree(p);
    delete h;
    return RT_OK;
}

rt_status rt_mlp_get_params(rt_mlp* h, float* params, float* ff) {
    if (!h || !params || !ff) return rt_internal_fail(RT_ERR_ARG, "NULL argument");
    hipStream_t s = rt_internal_stream(h->ctx);
    MLP_HIP(hipMemcpyAsync(params, h->params, h->lay.total * sizeof(float), hipMemcpyDeviceToDevice, s));
    MLP_HIP(hipMemcpyAsync(ff, h->ff, rt::kFreq * 5 * sizeof(float), hipMemcpyDeviceToDevice, s));
    return RT_OK;
}

rt_status rt_mlp_set_params(rt_mlp* h, const float* params, const float* ff) {
    if (!h || !params || !ff) return rt_internal_fail(RT_ERR_ARG, "NULL argument");
    hipStream_t s = rt_internal_stream(h->ctx);
    MLP_HIP(hipMemcpyAsync(h->params, params, h->lay.total * sizeof(float), hipMemcpyDeviceToDevice, s));
    MLP_HIP(hipMemcpyAsync(h->ff, ff, rt::kFreq * 5 * sizeof(float), hipMemcpyDeviceToDevice, s));
    MLP_HIP(hipMemsetAsync(h->m1, 0, h->lay.total * sizeof(float), s));
    MLP_HIP(hipMemsetAsync(h->m2, 0, h->lay.total * sizeof(float), s));
    h->step = 0;
    MLP_HIP(rt::launch_refresh_bf16(h->params, h->lay, h->wbf, h->wtbf, s));
    return RT_OK;
}

rt_status rt_mlp_forward(rt_mlp* h, const float* v, int64_t n, float* y) {
    if (!h || !v || !y) return rt_internal_fail(RT_ERR_ARG, "NULL argument");
    rt_status st = check_rows(h, n);
    if (st != RT_OK) return st;
    hipStream_t s = rt_internal_stream(h->ctx);
    MLP_HIP(hipSetDevice(rt_internal_device(h->ctx)));
    if ((st = forward(h, v, n, s)) != RT_OK) return st;
    const rt::MlpLayout& L = h->lay;
    MLP_HIP(rt::launch_head(h->H[3], h->Z[3], h->params + L.w_off[4], h->params + L.b_off[4], v, h->norm, nullptr,
                            nullptr, n, nullptr, y, nullptr, nullptr, nullptr, nullptr, s));
    return RT_OK;
}

rt_status rt_mlp_grad(rt_mlp* h, const float* v, const float* t, const float* m, int64_t n, float* grad,
                      float* loss) {
    if (!h || !v || !t || !m || !grad) return rt_internal_fail(RT_ERR_ARG, "NULL argument");
    rt_status st = check_rows(h, n);
    if (st != RT_OK) return st;
    hipStream_t s = rt_internal_stream(h->ctx);
    MLP_HIP(hipSetDevice(rt_internal_device(h->ctx)));
    if ((st = gradient(h, v, t, m, n, s)) != RT_OK) return st;
    MLP_HIP(hipMemcpyAsync(grad, h->grad, h->lay.total * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (loss) MLP_HIP(hipMemcpyAsync(loss, h->scal + 1, sizeof(float), hipMemcpyDeviceToDevice, s));
    return RT_OK;
}

rt_status rt_mlp_train_step(rt_mlp* h, const float* v, const float* t, const float* m, int64_t n, float lr,
                            float* loss) {
    if (!h || !v || !t || !m) return rt_internal_fail(RT_ERR_ARG, "NULL argument");
    if (!(lr > 0) || !std::isfinite(lr)) return rt_internal_fail(RT_ERR_ARG, "lr must be positive");
    rt_status st = check_rows(h, n);
    if (st != RT_OK) return st;
    hipStream_t s = rt_internal_stream(h->ctx);
    MLP_HIP(hipSetDevice(rt_internal_device(h->ctx)));
    if ((st = gradient(h, v, t, m, n, s)) != RT_OK) return st;
    h->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)h->step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)h->step)));
    MLP_HIP(rt::launch_adam(h->params, h->grad, h->m1, h->m2, h->lay.total, lr, b1, b2, 1e-8f, c1, c2, s));
    MLP_HIP(rt::launch_refresh_bf16(h->params, h->lay, h->wbf, h->wtbf, s));
    if (loss) MLP_HIP(hipMemcpyAsync(loss, h->scal + 1, sizeof(float), hipMemcpyDeviceToDevice, s));
    return RT_OK;
}

rt_status rt_mlp_valid_index(rt_mlp* h, const uint8_t* mask, int64_t n, uint32_t* index, int64_t capacity,
                             int64_t* count) {
    if (!h || !mask || !count || (capacity > 0 && !index)) return rt_internal_fail(RT_ERR_ARG, "NULL argument");
    if (n < 1 || n >= (int64_t(1) << 32)) return rt_internal_fail(RT_ERR_ARG, "mask length must be in [1, 2^32)");
    if (capacity < 0) return rt_internal_fail(RT_ERR_ARG, "negative capacity");
    hipStream_t s = rt_internal_stream(h->ctx);
    MLP_HIP(hipSetDevice(rt_internal_device(h->ctx)));
    const int64_t tiles = (n + rt::kIndexTile - 1) / rt::kIndexTile;
    uint32_t* cnt = nullptr;
    uint64_t* off = nullptr;
    MLP_HIP(hipMalloc((void**)&cnt, (size_t)tiles * sizeof(uint32_t)));
    hipError_t e = hipMalloc((void**)&off, (size_t)(tiles + 1) * sizeof(uint64_t));
    uint64_t total = 0;
    if (e == hipSuccess) e = rt::launch_index_count(mask, n, cnt, s);
    if (e == hipSuccess) e = rt::launch_index_scan(cnt, tiles, off, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&total, off + tiles, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && (int64_t)total <= capacity) e = rt::launch_index_write(mask, n, off, index, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(cnt);
    if (off) (void)hipFree(off);
    MLP_HIP(e);
    *count = (int64_t)total;
    if ((int64_t)total > capacity) return rt_internal_fail(RT_ERR_CAPACITY, "index capacity below the valid-cell count");
    return RT_OK;
}

rt_status rt_mlp_sample_batch(rt_mlp* h, const float* maps, const uint32_t* index, int64_t count, const float* tx,
                              int32_t T, const rt_grid* g, uint64_t seed, uint64_t step, float* v, float* t, float* m,
                              int64_t n) {
    if (!h || !maps || !index || !tx || !g || !v || !t || !m) return rt_internal_fail(RT_ERR_ARG, "NULL argument");
    if (T < 1 || n < 1 || g->nx < 1 || g->ny < 1) return rt_internal_fail(RT_ERR_ARG, "empty map stack or batch");
    if (count < 1) return rt_internal_fail(RT_ERR_ARG, "no usable cells (count < 1)");
    hipStream_t s = rt_internal_stream(h->ctx);
    MLP_HIP(rt::launch_sample(maps, index, count, tx, T, g->x0, g->y0, g->cell, g->nx, g->ny, seed, step, v, t, m, n,
                              s));
    return RT_OK;
}

rt_status rt_mlp_predict_maps(rt_mlp* h, const float* tx, int32_t T, const rt_grid* g, float* maps) {
    if (!h || !tx || !g || !maps) return rt_internal_fail(RT_ERR_ARG, "NULL argument");
    if (T < 1 || g->nx < 1 || g->ny < 1) return rt_internal_fail(RT_ERR_ARG, "empty map stack");
    if ((double)T * g->nx * g->ny >= 0x1p40) return rt_internal_fail(RT_ERR_ARG, "map stack of 2^40 cells or more");
    hipStream_t s = rt_internal_stream(h->ctx);
    MLP_HIP(hipSetDevice(rt_internal_device(h->ctx)));
    MLP_HIP(rt::launch_infer_v2(tx, T, g->x0, g->y0, g->cell, g->nx, g->ny, h->ff, h->norm, h->wfrag, h->lay,
                                h->params, maps, h->num_cu, s));
    return RT_OK;
}

rt_status rt_mlp_predict_maps_fallback(rt_mlp* h, rt_scene* scene, const rt_trace_params* p, const rt_device* tx,
                                       int32_t T, const rt_device* rx_ant, const rt_grid* g, const uint8_t* fallback,
                                       float* maps, int64_t* fallback_cells) {
    if (!h || !scene || !p || !tx || !rx_ant || !g || !fallback || !maps)
        return rt_internal_fail(RT_ERR_ARG, "NULL argument");
    if (rt_internal_scene_ctx(scene) != h->ctx)
        return rt_internal_fail(RT_ERR_ARG, "scene and surrogate belong to different contexts");
    if (T < 1 || g->nx < 1 || g->ny < 1) return rt_internal_fail(RT_ERR_ARG, "empty map stack");
    if ((double)T * g->nx * g->ny >= 0x1p40) return rt_internal_fail(RT_ERR_ARG, "map stack of 2^40 cells or more");
    for (int32_t k = 0; k < T; ++k)
        if (!std::isfinite(tx[k].pos[0]) || !std::isfinite(tx[k].pos[1]) || !std::isfinite(tx[k].pos[2]))
            return rt_internal_fail(RT_ERR_ARG, "a transmitter position is not finite");
    hipStream_t s = rt_internal_stream(h->ctx);
    MLP_HIP(hipSetDevice(rt_internal_device(h->ctx)));
    const size_t cells = (size_t)g->nx * g->ny;
    auto grow = [&](void** ptr, size_t& have, size_t want, size_t elem) -> hipError_t {
        if (have >= want && *ptr) return hipSuccess;
        if (*ptr) {
            const hipError_t e = hipFree(*ptr);
            if (e != hipSuccess) return e;
            *ptr = nullptr;
        }
        have = 0;
        const hipError_t e = hipMalloc(ptr, want * elem);
        if (e == hipSuccess) have = want;
        return e;
    };
    MLP_HIP(hipStreamSynchronize(s));  // earlier calls may still read the scratch being regrown
    MLP_HIP(grow((void**)&h->fb_tx, h->fb_tx_n, (size_t)T * 3, sizeof(float)));
    size_t cells_g = h->fb_cells, cells_h = h->fb_cells;
    MLP_HIP(grow((void**)&h->fb_gain, cells_g, cells, sizeof(float)));
    MLP_HIP(grow((void**)&h->fb_hits, cells_h, cells, sizeof(uint32_t)));
    h->fb_cells = std::min(cells_g, cells_h);
    if (!h->fb_count) MLP_HIP(hipMalloc((void**)&h->fb_count, sizeof(unsigned long long)));
    std::vector<float> pos(3 * (size_t)T);
    for (int32_t k = 0; k < T; ++k)
        for (int i = 0; i < 3; ++i) pos[3 * k + i] = tx[k].pos[i];
    MLP_HIP(hipMemcpyAsync(h->fb_tx, pos.data(), pos.size() * sizeof(float), hipMemcpyHostToDevice, s));
    // 1. the surrogate's maps
    MLP_HIP(rt::launch_infer_v2(h->fb_tx, T, g->x0, g->y0, g->cell, g->nx, g->ny, h->ff, h->norm, h->wfrag, h->lay,
                                h->params, maps, h->num_cu, s));
    // 2. how many cells fall back
    unsigned long long n = 0;
    MLP_HIP(hipMemsetAsync(h->fb_count, 0, sizeof(unsigned long long), s));
    MLP_HIP(rt::launch_count_u8(fallback, (int64_t)cells, h->fb_count, s));
    MLP_HIP(hipMemcpyAsync(&n, h->fb_count, sizeof(n), hipMemcpyDeviceToHost, s));
    MLP_HIP(hipStreamSynchronize(s));  // also ends the staging of pos
    if (fallback_cells) *fallback_cells = (int64_t)n;
    if (n == 0) return RT_OK;
    // 3. every transmitter's traced map, merged into the fallback cells
    for (int32_t k = 0; k < T; ++k) {
        const rt_status st = rt_coverage_map(h->ctx, scene, p, tx + k, rx_ant, g, h->fb_gain, h->fb_hits, nullptr,
                                             nullptr);
        if (st != RT_OK) return st;
        MLP_HIP(rt::launch_fallback_merge(fallback, h->fb_gain, (int64_t)cells, maps + (size_t)k * cells, s));
    }
    return RT_OK;
}

}  // extern "C"
