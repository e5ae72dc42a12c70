// Launch interface between the surrogate's C ABI (mlp_api.hip) and its
// kernels (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rt {

constexpr int kFreq = 64;
enum : int { kEpiStoreF32 = 0, kEpiBiasGelu = 1, kEpiGeluGrad = 2 };

struct GemmArgs {  // C[m][n] = sum_k A[m * lda + k] B[n * ldb + k], bf16 in, fp32 accumulate
    const __bf16* A;
    const __bf16* B;
    int lda, ldb;
    int M, N, K, ksplit;
    int epi;
    const float* bias;     // kEpiBiasGelu
    __bf16* outZ;          // kEpiBiasGelu: z; kEpiGeluGrad: dz (may be null for z)
    __bf16* outH;          // kEpiBiasGelu: gelu(z)
    const __bf16* Zprev;   // kEpiGeluGrad
    float* outF;           // kEpiStoreF32: [split][M][N]
};

struct MlpNorm {
    float center[5];
    float inv_half[5];
    // free-space prior added to the head: prior_db - 10 log10(d^2), d from the
    // transmitter to (cell x, cell y, prior_rx_z); prior_on = 0 disables it
    float prior_db;  // 20 log10(c0 / (4 pi f))
    float prior_rx_z;
    int32_t prior_on;
};

struct MlpLayout {
    int64_t w_off[5], w_size[5], b_off[5];
    int32_t fan_in[5];
    int64_t bf_off[4];
    int64_t total;
};

hipError_t launch_gemm_nt(const GemmArgs& g, int splits, hipStream_t s);
hipError_t launch_features(const float* v, int64_t n, const float* ff, const MlpNorm& norm, __bf16* out, hipStream_t s);
hipError_t launch_head(const __bf16* H4, const __bf16* Z4, const float* w5, const float* b5, const float* v,
                       const MlpNorm& norm, const float* t, const float* m, int64_t n, const float* msum, float* pred,
                       float* loss, __bf16* dZ4, float* gw5, float* gb5, hipStream_t s);
hipError_t launch_mask_sum(const float* m, int64_t n, float* out, hipStream_t s);
// *count += number of nonzero bytes of m[0 .. n) (count cleared by the caller).
hipError_t launch_count_u8(const uint8_t* m, int64_t n, unsigned long long* count, hipStream_t s);
// out[c] = 10 log10(gain[c]) (or -inf) for the cells with fallback[c] != 0.
hipError_t launch_fallback_merge(const uint8_t* fallback, const float* gain, int64_t n, float* out, hipStream_t s);
hipError_t launch_transpose(const __bf16* in, int64_t R, int64_t C, __bf16* out, hipStream_t s);
hipError_t launch_rowsum(const __bf16* dZt, int64_t rows, int64_t cols, float* db, hipStream_t s);
hipError_t launch_reduce_splits(const float* part, int S, int64_t n, float* grad, hipStream_t s);
// Fourier-matrix initialisation (see init_kernel).
struct MlpFourier {
    float s_tx, s_cell, s_rel;
    int32_t rows_tx, rows_rel;
};
hipError_t launch_mlp_init(float* params, float* ff, uint64_t seed, const MlpFourier& fs, const MlpLayout& lay,
                           hipStream_t s);
hipError_t launch_refresh_bf16(const float* params, const MlpLayout& lay, __bf16* wbf, __bf16* wtbf, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m1, float* m2, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);
hipError_t launch_sample(const float* maps, const uint32_t* index, int64_t count, const float* tx, int32_t T,
                         double gx0, double gy0, double gcell, int32_t gnx, int32_t gny, uint64_t seed, uint64_t step,
                         float* v, float* t, float* m, int64_t n, hipStream_t s);
// Ordered compaction of the nonzero positions of a byte mask: per-tile
// counts (tiles of kIndexTile entries), one-block exclusive scan of the tile
// counts (total in offsets[tiles]), then the ordered writes.
constexpr int kIndexTile = 4096;
hipError_t launch_index_count(const uint8_t* mask, int64_t n, uint32_t* tile_counts, hipStream_t s);
hipError_t launch_index_scan(const uint32_t* tile_counts, int64_t tiles, uint64_t* offsets, hipStream_t s);
hipError_t launch_index_write(const uint8_t* mask, int64_t n, const uint64_t* offsets, uint32_t* index,
                              hipStream_t s);
// Register-resident f16 map inference: fragment weights are rebuilt from
// the fp32 parameters into wfrag (v2_weights_halves() f16) on every call.
int64_t v2_weights_halves();
hipError_t launch_infer_v2(const float* tx, int32_t T, double gx0, double gy0, double gcell, int32_t gnx, int32_t gny,
                           const float* ff, const MlpNorm& norm, _Float16* wfrag, const MlpLayout& lay,
                           const float* params, float* out, int grid, hipStream_t s);
hipError_t launch_map_inputs(const float* tx, int32_t T, double gx0, double gy0, double gcell, int32_t gnx,
                             int32_t gny, int64_t row0, int64_t rows, float* v, hipStream_t s);

}  // namespace rt
