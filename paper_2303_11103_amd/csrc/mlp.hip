// Fourier-feature MLP surrogate of coverage maps for gfx950: bf16 MFMA
// training and inference kernels with fp32 accumulation.
//
// Network (see include/rt.h): v in R^5 (tx x, y, z, cell x, y, normalised)
// -> gamma(v) = [sin 2 pi B v, cos 2 pi B v] (B in R^{64x5}) -> 4 x (256,
// tanh-form GELU) -> linear head -> path gain in dB.  Loss: masked mean
// squared error in dB.  The paper gives no network (it motivates learned
// propagation models, Sec. I); the ray tracer supplies the training maps.
//
// All matrix products are one NT-GEMM kernel, C[m][n] = sum_k A[m][k] B[n][k]
// with k contiguous in both operands, on v_mfma_f32_16x16x32_bf16:
//   forward  H_l = gelu(H_{l-1} W_l^T + b_l)        A = H_{l-1}, B = W_l
//   backward dZ_{l-1} = (dZ_l W_l) * gelu'(Z_{l-1})  A = dZ_l,    B = W_l^T
//            dW_l = dZ_l^T H_{l-1} (split over rows) A = dZ_l^T,  B = H_{l-1}^T
// The transposed operands come from a tiled transpose kernel.
#include <hip/hip_runtime.h>

#include "mlp_kernels.h"

namespace rt {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

constexpr float kGeluC = 0.7978845608028654f;  // sqrt(2 / pi)

// tanh-form GELU written with the logistic function: 0.5 x (1 + tanh u) =
// x sigma(2u), u = sqrt(2/pi) (x + 0.044715 x^3); hardware exp and reciprocal.
__device__ __forceinline__ float sigm2(float u) { return __builtin_amdgcn_rcpf(1.0f + __expf(-2.0f * u)); }
__device__ __forceinline__ float gelu(float x) {
    const float u = kGeluC * (x + 0.044715f * x * x * x);
    return x * sigm2(u);
}
__device__ __forceinline__ float gelu_grad(float x) {
    const float u = kGeluC * (x + 0.044715f * x * x * x);
    const float s = sigm2(u);
    const float du = kGeluC * (1.0f + 3.0f * 0.044715f * x * x);
    return s + 2.0f * x * s * (1.0f - s) * du;
}

// Free-space gain [dB] of the link from the transmitter (v[0..2]) to the cell
// (v[3], v[4], prior_rx_z); 0 when the prior is off.
__device__ __forceinline__ float prior_db(const MlpNorm& nm, float tx, float ty, float tz, float cx, float cy) {
    if (!nm.prior_on) return 0.0f;
    const float dx = cx - tx, dy = cy - ty, dz = nm.prior_rx_z - tz;
    const float d2 = fmaxf(dx * dx + dy * dy + dz * dz, 1e-6f);
    return nm.prior_db - 3.0102999566398120f * __log2f(d2);  // 10 log10(d2) = (10 log10 2) log2(d2)
}

// ------------------------------------------------------------------ GEMM
constexpr int BM = 128, BN = 128, BK = 32, LDT = BK + 8;

__global__ __launch_bounds__(256) void gemm_nt_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) bf16 As[BM][LDT];
    __shared__ __attribute__((aligned(16))) bf16 Bs[BN][LDT];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int k_begin = blockIdx.z * g.ksplit;
    const int k_end = min(g.K, k_begin + g.ksplit);
    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = k_begin; k0 < k_end; k0 += BK) {
        for (int c = tid; c < BM * (BK / 8); c += 256) {
            const int r = c >> 2, kc = (c & 3) * 8;
            *reinterpret_cast<uint4*>(&As[r][kc]) =
                *reinterpret_cast<const uint4*>(g.A + (size_t)(m0 + r) * g.lda + k0 + kc);
            *reinterpret_cast<uint4*>(&Bs[r][kc]) =
                *reinterpret_cast<const uint4*>(g.B + (size_t)(n0 + r) * g.ldb + k0 + kc);
        }
        __syncthreads();
        bf16x8 af[4], bfr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            af[i] = *reinterpret_cast<const bf16x8*>(&As[wm * 64 + i * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn * 64 + j * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 64 + i * 16 + (lane >> 4) * 4 + r;
                const float v = acc[i][j][r];
                const size_t at = (size_t)row * g.N + col;
                if (g.epi == kEpiStoreF32) {
                    g.outF[(size_t)blockIdx.z * g.M * g.N + at] = v;
                } else if (g.epi == kEpiBiasGelu) {
                    const float z = v + g.bias[col];
                    g.outZ[at] = (bf16)z;
                    g.outH[at] = (bf16)gelu(z);
                } else {  // kEpiGeluGrad
                    const float zp = (float)g.Zprev[at];
                    g.outZ[at] = (bf16)(v * gelu_grad(zp));
                }
            }
        }
    }
}

// ------------------------------------------------------------------ elementwise
__global__ void features_kernel(const float* __restrict__ v, int64_t n, const float* __restrict__ ff,
                                MlpNorm norm, bf16* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * kFreq) return;
    const int64_t row = idx / kFreq;
    const int j = (int)(idx - row * kFreq);
    float rev = 0.0f;
    for (int i = 0; i < 5; ++i) rev += ff[j * 5 + i] * ((v[row * 5 + i] - norm.center[i]) * norm.inv_half[i]);
    float s, c;
    sincospif(2.0f * rev, &s, &c);
    out[row * (2 * kFreq) + j] = (bf16)s;
    out[row * (2 * kFreq) + kFreq + j] = (bf16)c;
}

// pred = w5 . h4 + b5; loss and dZ4 = g w5 gelu'(Z4); dw5 and db5 partial sums.
__global__ __launch_bounds__(256) void head_kernel(const bf16* __restrict__ H4, const bf16* __restrict__ Z4,
                                                   const float* __restrict__ w5, const float* __restrict__ b5,
                                                   const float* __restrict__ v, MlpNorm norm,
                                                   const float* __restrict__ t, const float* __restrict__ m,
                                                   int64_t n, const float* __restrict__ msum, float* __restrict__ pred,
                                                   float* __restrict__ loss, bf16* __restrict__ dZ4,
                                                   float* __restrict__ gw5, float* __restrict__ gb5) {
    __shared__ float sw[256];
    __shared__ float sg[256];
    __shared__ float acc[256];
    const int tid = threadIdx.x;
    sw[tid] = w5[tid];
    acc[tid] = 0.0f;
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * 256;
    // one thread per row: prediction and dL/dy
    {
        const int64_t row = r0 + tid;
        float gval = 0.0f;
        if (row < n) {
            float y = b5[0];
            for (int k = 0; k < 256; ++k) y += sw[k] * (float)H4[row * 256 + k];
            const float* vr = v + 5 * row;
            y += prior_db(norm, vr[0], vr[1], vr[2], vr[3], vr[4]);
            if (pred) pred[row] = y;
            if (t) {
                const float inv = 1.0f / fmaxf(msum[0], 1.0f);
                const float e = y - t[row];
                gval = 2.0f * m[row] * e * inv;
                atomicAdd(loss, m[row] * e * e * inv);
            }
        }
        sg[tid] = gval;
    }
    __syncthreads();
    if (!t) return;
    if (tid == 0) {
        float s = 0.0f;
        for (int i = 0; i < 256; ++i) s += sg[i];
        atomicAdd(gb5, s);
    }
    // thread = feature column k: dw5[k] += sum_rows g h4[row][k]; dZ4 = g w5[k] gelu'(z)
    const int k = tid;
    float a = 0.0f;
    for (int i = 0; i < 256; ++i) {
        const int64_t row = r0 + i;
        if (row >= n) break;
        const float gi = sg[i];
        a += gi * (float)H4[row * 256 + k];
        dZ4[row * 256 + k] = (bf16)(gi * sw[k] * gelu_grad((float)Z4[row * 256 + k]));
    }
    atomicAdd(gw5 + k, a);
}

__global__ void mask_sum_kernel(const float* __restrict__ m, int64_t n, float* __restrict__ out) {
    __shared__ float s[256];
    float a = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a += m[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, s[0]);
}

// out[c][r] = in[r][c] for an R x C bf16 matrix (R, C multiples of 32)
__global__ void transpose_kernel(const bf16* __restrict__ in, int64_t R, int64_t C, bf16* __restrict__ out) {
    __shared__ bf16 tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    for (int i = threadIdx.y; i < 32; i += 8) tile[i][threadIdx.x] = in[(r0 + i) * C + c0 + threadIdx.x];
    __syncthreads();
    for (int i = threadIdx.y; i < 32; i += 8) out[(c0 + i) * R + r0 + threadIdx.x] = tile[threadIdx.x][i];
}

// db[n] += sum_rows dZ[row][n] (dZ: rows x N, N = 256)
__global__ void colsum_kernel(const bf16* __restrict__ dZ, int64_t rows, float* __restrict__ db) {
    const int n = threadIdx.x;
    float a = 0.0f;
    const int64_t r0 = (int64_t)blockIdx.x * 256;
    for (int64_t i = r0; i < r0 + 256 && i < rows; ++i) a += (float)dZ[i * 256 + n];
    atomicAdd(db + n, a);
}

// grad[i] += sum_s part[s][i]
__global__ void reduce_splits_kernel(const float* __restrict__ part, int S, int64_t n, float* __restrict__ grad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float a = 0.0f;
    for (int s = 0; s < S; ++s) a += part[(int64_t)s * n + i];
    grad[i] += a;
}

__device__ __forceinline__ uint64_t splitmix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__device__ __forceinline__ float u01(uint64_t h) { return ((float)(h >> 40) + 0.5f) * 0x1p-24f; }

// Weights uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)), biases 0; Fourier matrix
// N(0, s^2) with s = ff_scale_tx on the transmitter columns (0..2) and
// ff_scale_cell on the cell columns (3, 4).
__global__ void init_kernel(float* __restrict__ params, float* __restrict__ ff, uint64_t seed, float ff_scale_tx,
                            float ff_scale_cell, MlpLayout lay) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < lay.total) {
        float v = 0.0f;
        for (int l = 0; l < 5; ++l) {
            if (i >= lay.w_off[l] && i < lay.w_off[l] + lay.w_size[l]) {
                const float bound = rsqrtf((float)lay.fan_in[l]);
                v = (2.0f * u01(splitmix(seed ^ (uint64_t)i)) - 1.0f) * bound;
            }
        }
        params[i] = v;
    }
    if (i < kFreq * 5) {
        const uint64_t h1 = splitmix(seed * 7919u + 0x1234567ull + 2 * (uint64_t)i);
        const uint64_t h2 = splitmix(seed * 7919u + 0x1234567ull + 2 * (uint64_t)i + 1);
        const float r = sqrtf(-2.0f * logf(u01(h1)));
        ff[i] = ((i % 5) < 3 ? ff_scale_tx : ff_scale_cell) * r * cospif(2.0f * u01(h2));
    }
}

// bf16 copies: W_l [out][in] and W_l^T [in][out]
__global__ void refresh_bf16_kernel(const float* __restrict__ params, MlpLayout lay, bf16* __restrict__ wbf,
                                    bf16* __restrict__ wtbf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int l = 0; l < 4; ++l) {
        const int64_t sz = lay.w_size[l];
        if (i < sz) {
            const int fan = lay.fan_in[l];
            const int64_t o = i / fan, k = i - o * fan;
            const bf16 b = (bf16)params[lay.w_off[l] + i];
            wbf[lay.bf_off[l] + i] = b;
            wtbf[lay.bf_off[l] + k * 256 + o] = b;
        }
    }
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                            float* __restrict__ m2, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    p[i] -= lr * (a * c1) / (sqrtf(b * c2) + eps);
}

// Random (tx, cell) samples from a stack of maps: counter-based hash of
// (seed, step, row); up to 8 draws until a masked-in cell is found.
__global__ void sample_kernel(const float* __restrict__ maps, const uint32_t* __restrict__ index, int64_t count,
                              const float* __restrict__ tx, int32_t T, double gx0, double gy0, double gcell,
                              int32_t gnx, int32_t gny, uint64_t seed, uint64_t step, float* __restrict__ v,
                              float* __restrict__ t, float* __restrict__ m, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t cells = (int64_t)gnx * gny;
    const uint64_t h = splitmix(seed ^ splitmix(step * 0x100000001B3ull + (uint64_t)i));
    const uint64_t s = index[h % (uint64_t)count];
    if (s >= (uint64_t)T * (uint64_t)cells) {  // an index that does not belong to this map stack
        for (int k = 0; k < 5; ++k) v[5 * i + k] = 0.0f;
        t[i] = 0.0f;
        m[i] = 0.0f;
        return;
    }
    const int64_t tt = (int64_t)(s / (uint64_t)cells), c = (int64_t)(s % (uint64_t)cells);
    const int64_t iy = c / gnx, ix = c - iy * gnx;
    v[5 * i + 0] = tx[3 * tt];
    v[5 * i + 1] = tx[3 * tt + 1];
    v[5 * i + 2] = tx[3 * tt + 2];
    v[5 * i + 3] = (float)(gx0 + (ix + 0.5) * gcell);
    v[5 * i + 4] = (float)(gy0 + (iy + 0.5) * gcell);
    t[i] = maps[s];
    m[i] = 1.0f;
}

// ------------------------------------------------------------------ valid-cell index
// 256 threads per tile of kIndexTile bytes; thread j owns bytes [16 j, 16 j + 16).
__device__ __forceinline__ uint32_t count16(const uint8_t* __restrict__ mask, int64_t b, int64_t n) {
    uint32_t c = 0;
    for (int k = 0; k < 16; ++k)
        if (b + k < n) c += mask[b + k] != 0;
    return c;
}

__global__ __launch_bounds__(256) void index_count_kernel(const uint8_t* __restrict__ mask, int64_t n,
                                                          uint32_t* __restrict__ tile_counts) {
    __shared__ uint32_t part[4];
    const int64_t b = (int64_t)blockIdx.x * kIndexTile + threadIdx.x * 16;
    uint32_t c = count16(mask, b, n);
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) tile_counts[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// one block of 1024 threads: exclusive prefix of the tile counts, total last
__global__ __launch_bounds__(1024) void index_scan_kernel(const uint32_t* __restrict__ cnt, int64_t tiles,
                                                          uint64_t* __restrict__ off) {
    __shared__ uint64_t wsum[16];
    __shared__ uint64_t carry;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < tiles; base += 1024) {
        const int64_t i = base + tid;
        const uint64_t x = i < tiles ? cnt[i] : 0;
        uint64_t incl = x;
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        uint64_t before = carry;
        for (int k = 0; k < w; ++k) before += wsum[k];
        if (i < tiles) off[i] = before + incl - x;
        __syncthreads();
        if (tid == 1023) carry = before + incl;
        __syncthreads();
    }
    if (tid == 0) off[tiles] = carry;
}

__global__ __launch_bounds__(256) void index_write_kernel(const uint8_t* __restrict__ mask, int64_t n,
                                                          const uint64_t* __restrict__ off,
                                                          uint32_t* __restrict__ index) {
    __shared__ uint32_t wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t b = (int64_t)blockIdx.x * kIndexTile + tid * 16;
    const uint32_t c = count16(mask, b, n);
    uint32_t incl = c;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint64_t at = off[blockIdx.x] + incl - c;
    for (int k = 0; k < w; ++k) at += wsum[k];
    for (int k = 0; k < 16; ++k)
        if (b + k < n && mask[b + k]) index[at++] = (uint32_t)(b + k);
}

// Inputs of every (tx, cell) pair of a map stack, rows ordered [tx][cell].
__global__ void map_inputs_kernel(const float* __restrict__ tx, int32_t T, double gx0, double gy0, double gcell,
                                  int32_t gnx, int32_t gny, int64_t row0, int64_t rows, float* __restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    const int64_t r = row0 + i;
    const int64_t cells = (int64_t)gnx * gny;
    const int64_t tt = r / cells, c = r - tt * cells;
    const int64_t iy = c / gnx, ix = c - iy * gnx;
    v[5 * i + 0] = tx[3 * tt];
    v[5 * i + 1] = tx[3 * tt + 1];
    v[5 * i + 2] = tx[3 * tt + 2];
    v[5 * i + 3] = (float)(gx0 + (ix + 0.5) * gcell);
    v[5 * i + 4] = (float)(gy0 + (iy + 0.5) * gcell);
}

// Fused inference over map rows (tx, cell): a block of 8 waves owns 128 rows;
// the activations stay in LDS across the four layers (one 128 x 256 bf16
// buffer, overwritten in place after a barrier), the weights stream from L2
// as MFMA B-fragments, wave w computes rows (w / 4) * 64 .. +64 and columns
// (w % 4) * 64 .. +64 of every layer, and the head reduces each row in four
// lanes.
constexpr int kInferRows = 128;
constexpr int kActLd = 256 + 8;

struct InferArgs {
    const float* tx;
    int32_t T;
    double gx0, gy0, gcell;
    int32_t gnx, gny;
    int64_t total;
    const float* ff;
    MlpNorm norm;
    const bf16* wbf;
    MlpLayout lay;
    const float* params;
    float* out;
};

__global__ __launch_bounds__(512) void infer_fused_kernel(InferArgs a) {
    __shared__ __attribute__((aligned(16))) bf16 act[kInferRows][kActLd];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rh = wave >> 2, cq = wave & 3;
    const int64_t row0 = (int64_t)blockIdx.x * kInferRows;
    const int64_t cells = (int64_t)a.gnx * a.gny;
    // Fourier features of the block's rows
    for (int e = tid; e < kInferRows * kFreq; e += 512) {
        const int r = e / kFreq, j = e - r * kFreq;
        int64_t gr = row0 + r;
        if (gr >= a.total) gr = a.total - 1;
        const int64_t t = gr / cells, c = gr - t * cells;
        const int64_t iy = c / a.gnx, ix = c - iy * a.gnx;
        const float v[5] = {a.tx[3 * t], a.tx[3 * t + 1], a.tx[3 * t + 2], (float)(a.gx0 + (ix + 0.5) * a.gcell),
                            (float)(a.gy0 + (iy + 0.5) * a.gcell)};
        float rev = 0.0f;
#pragma unroll
        for (int i = 0; i < 5; ++i) rev += a.ff[j * 5 + i] * ((v[i] - a.norm.center[i]) * a.norm.inv_half[i]);
        float sn, cs;
        sincospif(2.0f * rev, &sn, &cs);
        act[r][j] = (bf16)sn;
        act[r][kFreq + j] = (bf16)cs;
    }
    __syncthreads();
    for (int l = 0; l < 4; ++l) {
        const int K = a.lay.fan_in[l];
        const bf16* W = a.wbf + a.lay.bf_off[l];
        floatx4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        bf16x8 bn[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            bn[j] = *reinterpret_cast<const bf16x8*>(W + (size_t)(cq * 64 + j * 16 + (lane & 15)) * K + (lane >> 4) * 8);
        for (int k0 = 0; k0 < K; k0 += 32) {
            bf16x8 bc[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) bc[j] = bn[j];
            if (k0 + 32 < K) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    bn[j] = *reinterpret_cast<const bf16x8*>(W + (size_t)(cq * 64 + j * 16 + (lane & 15)) * K + k0 + 32 +
                                                             (lane >> 4) * 8);
            }
            bf16x8 af[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                af[i] = *reinterpret_cast<const bf16x8*>(&act[rh * 64 + i * 16 + (lane & 15)][k0 + (lane >> 4) * 8]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bc[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();  // every wave has read this layer's input
        const float* bias = a.params + a.lay.b_off[l];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = cq * 64 + j * 16 + (lane & 15);
            const float b = bias[col];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) act[rh * 64 + i * 16 + (lane >> 4) * 4 + r][col] = (bf16)gelu(acc[i][j][r] + b);
        }
        __syncthreads();
    }
    // head: four lanes per row
    const int r = tid >> 2, part = tid & 3;
    const float* w5 = a.params + a.lay.w_off[4];
    float y = 0.0f;
    for (int k = part * 64; k < part * 64 + 64; ++k) y += w5[k] * (float)act[r][k];
    y += __shfl_xor(y, 1);
    y += __shfl_xor(y, 2);
    const int64_t gr = row0 + r;
    if (part == 0 && gr < a.total) {
        const int64_t t = gr / cells, c = gr - t * cells;
        const int64_t iy = c / a.gnx, ix = c - iy * a.gnx;
        const float pr = prior_db(a.norm, a.tx[3 * t], a.tx[3 * t + 1], a.tx[3 * t + 2],
                                  (float)(a.gx0 + (ix + 0.5) * a.gcell), (float)(a.gy0 + (iy + 0.5) * a.gcell));
        a.out[gr] = y + a.params[a.lay.b_off[4]] + pr;
    }
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_gemm_nt(const GemmArgs& g, int splits, hipStream_t s) {
    if (g.M % BM || g.N % BN || g.K % BK || g.ksplit % BK) return hipErrorInvalidValue;
    dim3 grid(g.N / BN, g.M / BM, splits);
    hipLaunchKernelGGL(gemm_nt_kernel, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_features(const float* v, int64_t n, const float* ff, const MlpNorm& norm, bf16* out, hipStream_t s) {
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for(n * kFreq, 256)), dim3(256), 0, s, v, n, ff, norm, out);
    return hipGetLastError();
}

hipError_t launch_head(const bf16* H4, const bf16* Z4, const float* w5, const float* b5, const float* v,
                       const MlpNorm& norm, const float* t, const float* m, int64_t n, const float* msum, float* pred,
                       float* loss, bf16* dZ4, float* gw5, float* gb5, hipStream_t s) {
    hipLaunchKernelGGL(head_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, H4, Z4, w5, b5, v, norm, t, m, n, msum,
                       pred, loss, dZ4, gw5, gb5);
    return hipGetLastError();
}

hipError_t launch_mask_sum(const float* m, int64_t n, float* out, hipStream_t s) {
    hipLaunchKernelGGL(mask_sum_kernel, dim3(64), dim3(256), 0, s, m, n, out);
    return hipGetLastError();
}

hipError_t launch_transpose(const bf16* in, int64_t R, int64_t C, bf16* out, hipStream_t s) {
    if (R % 32 || C % 32) return hipErrorInvalidValue;
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)(C / 32), (unsigned)(R / 32)), dim3(32, 8), 0, s, in, R, C,
                       out);
    return hipGetLastError();
}

hipError_t launch_colsum(const bf16* dZ, int64_t rows, float* db, hipStream_t s) {
    hipLaunchKernelGGL(colsum_kernel, dim3(blocks_for(rows, 256)), dim3(256), 0, s, dZ, rows, db);
    return hipGetLastError();
}

hipError_t launch_reduce_splits(const float* part, int S, int64_t n, float* grad, hipStream_t s) {
    hipLaunchKernelGGL(reduce_splits_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, part, S, n, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_init(float* params, float* ff, uint64_t seed, float ff_scale_tx, float ff_scale_cell,
                           const MlpLayout& lay, hipStream_t s) {
    hipLaunchKernelGGL(init_kernel, dim3(blocks_for(lay.total, 256)), dim3(256), 0, s, params, ff, seed, ff_scale_tx,
                       ff_scale_cell, lay);
    return hipGetLastError();
}

hipError_t launch_refresh_bf16(const float* params, const MlpLayout& lay, bf16* wbf, bf16* wtbf, hipStream_t s) {
    hipLaunchKernelGGL(refresh_bf16_kernel, dim3(blocks_for(256 * 256, 256)), dim3(256), 0, s, params, lay, wbf, wtbf);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m1, float* m2, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, g, m1, m2, n, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}

hipError_t launch_sample(const float* maps, const uint32_t* index, int64_t count, const float* tx, int32_t T,
                         double gx0, double gy0, double gcell, int32_t gnx, int32_t gny, uint64_t seed, uint64_t step,
                         float* v, float* t, float* m, int64_t n, hipStream_t s) {
    if (count < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sample_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, maps, index, count, tx, T, gx0, gy0,
                       gcell, gnx, gny, seed, step, v, t, m, n);
    return hipGetLastError();
}

hipError_t launch_index_count(const uint8_t* mask, int64_t n, uint32_t* tile_counts, hipStream_t s) {
    hipLaunchKernelGGL(index_count_kernel, dim3(blocks_for(n, kIndexTile)), dim3(256), 0, s, mask, n, tile_counts);
    return hipGetLastError();
}

hipError_t launch_index_scan(const uint32_t* tile_counts, int64_t tiles, uint64_t* offsets, hipStream_t s) {
    hipLaunchKernelGGL(index_scan_kernel, dim3(1), dim3(1024), 0, s, tile_counts, tiles, offsets);
    return hipGetLastError();
}

hipError_t launch_index_write(const uint8_t* mask, int64_t n, const uint64_t* offsets, uint32_t* index,
                              hipStream_t s) {
    hipLaunchKernelGGL(index_write_kernel, dim3(blocks_for(n, kIndexTile)), dim3(256), 0, s, mask, n, offsets, index);
    return hipGetLastError();
}

hipError_t launch_infer_fused(const float* tx, int32_t T, double gx0, double gy0, double gcell, int32_t gnx,
                              int32_t gny, const float* ff, const MlpNorm& norm, const __bf16* wbf,
                              const MlpLayout& lay, const float* params, float* out, hipStream_t s) {
    InferArgs a;
    a.tx = tx;
    a.T = T;
    a.gx0 = gx0;
    a.gy0 = gy0;
    a.gcell = gcell;
    a.gnx = gnx;
    a.gny = gny;
    a.total = (int64_t)T * gnx * gny;
    a.ff = ff;
    a.norm = norm;
    a.wbf = wbf;
    a.lay = lay;
    a.params = params;
    a.out = out;
    hipLaunchKernelGGL(infer_fused_kernel, dim3(blocks_for(a.total, kInferRows)), dim3(512), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_map_inputs(const float* tx, int32_t T, double gx0, double gy0, double gcell, int32_t gnx,
                             int32_t gny, int64_t row0, int64_t rows, float* v, hipStream_t s) {
    hipLaunchKernelGGL(map_inputs_kernel, dim3(blocks_for(rows, 256)), dim3(256), 0, s, tx, T, gx0, gy0, gcell, gnx,
                       gny, row0, rows, v);
    return hipGetLastError();
}

}  // namespace rt
