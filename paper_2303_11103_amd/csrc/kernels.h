// Launch interface between the C ABI (api.hip) and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "device.h"
#include "layout.h"

namespace rt {

// State of one live ray between two bounces (96 bytes, read/written coalesced
// by consecutive lanes).
struct alignas(16) RayState {
    double o[3];    // origin (fp64)
    double d[3];    // unit direction (fp64)
    float E[6];     // field, complex Cartesian (re, im) per axis
    int32_t excl;   // face of the last reflection (-1 at the transmitter)
    int32_t prefix; // candidate-table slot of the face sequence so far (-1 none)
    int32_t ray;    // lattice position j: ray index = begin + j * stride
    int32_t pad;
};
static_assert(sizeof(RayState) == 96, "ray state size");

constexpr uint64_t kEmptyKey = ~0ull;
constexpr int kQueueRegions = 64;

struct DevScene {
    const Node* nodes;
    const Tri* tris;
    const Shade* shades;
    const Face* faces;
    const int32_t* face_tris;
    int32_t num_faces;
    int32_t nt;
    int32_t num_nodes;
    int32_t pad;
};

struct SbrArgs {
    DevScene sc;
    int64_t num_rays;   // lattice size N
    int64_t begin, stride;
    int64_t count;      // traced rays (positions 0..count-1)
    int64_t pos0, chunk; // positions handled by this launch sequence: [pos0, pos0 + chunk)
    int64_t perm_f, perm_g;  // band permutation (Fibonacci numbers F_m, F_{m-1}); 0 = identity
    int64_t perm_full;       // positions below this are permuted (whole bands)
    double perm_inv;         // 1 / F_m
    double tmin;
    double tx[3];
    Antenna tx_ant, rx_ant;
    // coverage
    double gx0, gy0, gcell, gz;
    int32_t gnx, gny;
    float wscale;       // (lambda/4pi)^2 (4pi/N) / cell^2
    float* gain;
    uint32_t* hits;
    // queues
    int32_t depth, max_depth;
    // The queues are split into kQueueRegions regions of region_cap rays; a
    // wave appends its survivors to region (wave % kQueueRegions) through
    // that region's counter, which spreads the queue atomics over 64 addresses.
    const RayState* in;
    const uint32_t* in_count;   // [kQueueRegions] counts of the input regions
    RayState* out;
    uint32_t* out_count;        // [kQueueRegions]
    int64_t region_cap;
    uint64_t* stats;    // [max_depth + 1] traced rays per depth (nullable)
    uint64_t* work;     // stats mode: [3][max_depth + 1] rays, inner-node visits, triangle tests
    // record mode
    int32_t* rec_tri;
    double* rec_t;
    // candidate mode
    uint64_t* table;
    uint64_t table_mask;
    uint32_t* overflow;
};

enum : int { kModeCoverage = 1, kModeRecord = 2, kModeCandidates = 4, kModeStats = 8 };

// Rays one queue region must hold for a bounce launch of `grid` blocks over
// at most `chunk` rays: the waves of a region (every kQueueRegions-th) times
// their grid-stride iterations times 64 lanes.
int64_t sbr_region_capacity(int64_t chunk, int grid);
hipError_t launch_sbr_bounce(const SbrArgs& a, const MatTable& mats, int mode, int grid, hipStream_t s);
hipError_t launch_fib_dirs(int64_t N, int64_t begin, int64_t stride, int64_t count, double* out, hipStream_t s);
hipError_t launch_finalize_db(const float* gain, float* db, int64_t n, hipStream_t s);

// ---------------------------------------------------------------- paths
struct Cand {
    int32_t depth;
    int32_t faces[8];
};

struct PathArgs {
    DevScene sc;
    double freq, lambda;
    double tx[3];
    Antenna tx_ant;
    const double* rx;        // [nrx][3]
    const Antenna* rx_ant;   // [nrx]
    int32_t nrx;
    const Cand* cands;
    const uint32_t* ncand;   // device count
    int32_t max_depth;
    int32_t P;               // slots per rx
    uint32_t* counts;        // [nrx] paths found
    // unsorted path records
    float* a;      // [nrx][P][2]
    float* T;      // [nrx][P][8]
    float* tau;    // [nrx][P]
    float* aod;    // [nrx][P][2]
    float* aoa;    // [nrx][P][2]
    int32_t* depth;   // [nrx][P]
    int32_t* faces;   // [nrx][P][FD]
    int32_t fd;       // faces stride = max(max_depth, 1)
};

hipError_t launch_paths_power(const float* a, const int32_t* depth, int64_t n, int P, double* power, hipStream_t s);
hipError_t launch_extract_candidates(const uint64_t* table, uint64_t cap, int32_t max_depth, Cand* out,
                                     uint32_t* count, uint32_t max_out, hipStream_t s);
hipError_t launch_image_paths(const PathArgs& a, const MatTable& mats, int64_t max_items, hipStream_t s);
hipError_t launch_sort_paths(const PathArgs& a, int32_t nrx, float* a_out, float* T_out, float* tau_out,
                             float* aod_out, float* aoa_out, int32_t* depth_out, int32_t* faces_out,
                             int32_t* num_paths_out, hipStream_t s);

struct GradArgs {
    DevScene sc;
    double freq, lambda;
    double tx[3];
    double yaw, pitch, roll;
    int32_t tx_pattern;
    const double* rx;
    const Antenna* rx_ant;
    int32_t nrx, P, fd;
    const int32_t* depth;   // [nrx][P]
    const int32_t* faces;   // [nrx][P][fd]
    const double* dL_dP;    // [nrx]
    double* grad;           // [2 nm + 5]
    int32_t nm;
};
hipError_t launch_power_grad(const GradArgs& a, const MatTable& mats, hipStream_t s);


// ---------------------------------------------------------------- MLP surrogate
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
};

struct MlpLayout {
    int64_t w_off[5], w_size[5], b_off[5];
    int32_t fan_in[5];
    int64_t bf_off[4];
    int64_t total;
};

hipError_t launch_gemm_nt(const GemmArgs& g, int splits, hipStream_t s);
hipError_t launch_features(const float* v, int64_t n, const float* ff, const MlpNorm& norm, __bf16* out, hipStream_t s);
hipError_t launch_head(const __bf16* H4, const __bf16* Z4, const float* w5, const float* b5, const float* t,
                       const float* m, int64_t n, const float* msum, float* pred, float* loss, __bf16* dZ4, float* gw5,
                       float* gb5, hipStream_t s);
hipError_t launch_mask_sum(const float* m, int64_t n, float* out, hipStream_t s);
hipError_t launch_transpose(const __bf16* in, int64_t R, int64_t C, __bf16* out, hipStream_t s);
hipError_t launch_colsum(const __bf16* dZ, int64_t rows, float* db, hipStream_t s);
hipError_t launch_reduce_splits(const float* part, int S, int64_t n, float* grad, hipStream_t s);
hipError_t launch_mlp_init(float* params, float* ff, uint64_t seed, float ff_scale, const MlpLayout& lay,
                           hipStream_t s);
hipError_t launch_refresh_bf16(const float* params, const MlpLayout& lay, __bf16* wbf, __bf16* wtbf, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m1, float* m2, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);
hipError_t launch_sample(const float* maps, const uint8_t* mask, const float* tx, int32_t T, double gx0, double gy0,
                         double gcell, int32_t gnx, int32_t gny, uint64_t seed, uint64_t step, float* v, float* t,
                         float* m, int64_t n, hipStream_t s);
hipError_t launch_infer_fused(const float* tx, int32_t T, double gx0, double gy0, double gcell, int32_t gnx,
                              int32_t gny, const float* ff, const MlpNorm& norm, const __bf16* wbf,
                              const MlpLayout& lay, const float* params, float* out, hipStream_t s);
hipError_t launch_map_inputs(const float* tx, int32_t T, double gx0, double gy0, double gcell, int32_t gnx,
                             int32_t gny, int64_t row0, int64_t rows, float* v, hipStream_t s);

}  // namespace rt
