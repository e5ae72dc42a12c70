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

#include <algorithm>

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
                acc[tid] = m[row] * e * e * inv;  // this row's share of the loss
            }
        }
        sg[tid] = gval;
    }
    __syncthreads();
    if (!t) return;
    if (tid == 0) {
        float s = 0.0f, l = 0.0f;
        for (int i = 0; i < 256; ++i) {
            s += sg[i];
            l += acc[i];
        }
        atomicAdd(gb5, s);
        atomicAdd(loss, l);  // one atomic per block
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
// db[c] += sum_i dZt[c][i]: one block per row c of the transposed gradient
// (contiguous), a tree reduction, no atomics.
__global__ __launch_bounds__(256) void rowsum_kernel(const bf16* __restrict__ dZt, int64_t cols,
                                                     float* __restrict__ db) {
    __shared__ float part[4];
    const bf16* p = dZt + (int64_t)blockIdx.x * cols;
    float a = 0.0f;
    for (int64_t i = threadIdx.x; i < cols; i += 256) a += (float)p[i];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) db[blockIdx.x] += part[0] + part[1] + part[2] + part[3];
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

// Weights uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)), biases 0.  Fourier matrix
// (64 x 5, columns tx x, y, z, cell x, y) from unit normals z(f, c):
// independent (rows_tx = rows_rel = 0): s_tx z on the transmitter columns,
// s_cell z on the cell columns; structured: rows f < rows_tx transmitter only
// (s_tx z), rows f >= 64 - rows_rel the cell relative to the transmitter
// (s_rel z(f, 3..4) on the cell columns, the negatives on tx x, y, s_tx z on
// tx z), the rows between cell only (s_cell z).
__device__ __forceinline__ float unit_normal(uint64_t seed, int64_t i) {
    const uint64_t h1 = splitmix(seed * 7919u + 0x1234567ull + 2 * (uint64_t)i);
    const uint64_t h2 = splitmix(seed * 7919u + 0x1234567ull + 2 * (uint64_t)i + 1);
    return sqrtf(-2.0f * logf(u01(h1))) * cospif(2.0f * u01(h2));
}

__global__ void init_kernel(float* __restrict__ params, float* __restrict__ ff, uint64_t seed, MlpFourier fs,
                            MlpLayout lay) {
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
        const int f = (int)(i / 5), c = (int)(i % 5);
        const float z = unit_normal(seed, i);
        float b;
        if (fs.rows_tx + fs.rows_rel == 0) {
            b = (c < 3 ? fs.s_tx : fs.s_cell) * z;
        } else if (f < fs.rows_tx) {
            b = c < 3 ? fs.s_tx * z : 0.0f;
        } else if (f >= kFreq - fs.rows_rel) {
            if (c >= 3) b = fs.s_rel * z;
            else if (c == 2) b = fs.s_tx * z;
            else b = -fs.s_rel * unit_normal(seed, (int64_t)f * 5 + 3 + c);  // minus the cell entry
        } else {
            b = c >= 3 ? fs.s_cell * z : 0.0f;
        }
        ff[i] = b;
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

// ------------------------------------------------------------------ map inference (register-resident)
// Map inference with f16 MFMA (v_mfma_f32_16x16x32_f16), written as
// C = W X^T so that rows are the MFMA's n dimension: a wave keeps 32 rows (two
// n-tiles) of activations in registers for the whole network.  The output
// tile layout (lane l: features 4 (l / 16) + r of row l % 16) is the next
// layer's B operand once the k positions of a 32-feature step are mapped to
// features p -> p < 4 ? 4 g + p : 16 + 4 g + p - 4 (g = l / 16); the weights
// are pre-arranged with the same map, as 1 KB fragments (one per m-tile and
// k-step, 16 bytes per lane) that a block stages layer by layer in LDS.
// GELU (the tanh form) is evaluated in packed f16 as x clamp(1/2 + u Q(u^2),
// 0, 1), u = clamp(x / 4, -1, 1), Q a degree-6 least-squares fit (largest
// deviation 2e-4 in exact arithmetic); the factor 1/4 is folded into the
// weights and biases, so each layer's accumulators hold u and it passes on
// gelu / 4.  The Fourier features use the hardware sine and cosine of the
// phase in turns.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __fp16 fp16x2 __attribute__((ext_vector_type(2)));
constexpr int kV2Waves = 8;                 // 512 threads, 32 rows per wave
constexpr int kV2Rows = 32 * kV2Waves;      // rows per block pass
constexpr int kFragHalves = 512;            // 16 x 32 f16 per fragment
constexpr int kL1Frags = 16 * 4, kLFrags = 16 * 8;

struct InferV2Args {
    const float* tx;
    int32_t T;
    double gx0, gy0, gcell;
    int32_t gnx, gny;
    int64_t total;
    const float* ff;
    MlpNorm norm;
    const _Float16* wfrag;  // layer 1: kL1Frags fragments, layers 2..4: kLFrags each
    const float* params;
    MlpLayout lay;
    float* out;
};

// Two independent GELU pairs evaluated in lockstep: each step of one chain
// fills the slot that a dependent packed instruction of the other must wait.
// In: u = x / 4; out: gelu(x) / 4 = u clamp(1/2 + u Q(min(u^2, 1)), 0, 1).  For
// |u| > 1 the value 1/2 + u Q(1) lies outside [0, 1] (Q(1) > 1/2), so the
// clamp gives 0 or 1 exactly as with u clamped to [-1, 1].  Both clamps to
// [0, 1] become the instructions' clamp bits.
__device__ __forceinline__ void gelu2x2(f16x2& u0, f16x2& u1) {
    auto c = [](float v) { return (f16x2){(_Float16)v, (_Float16)v}; };
    auto clamp01 = [](f16x2 v) {
        return __builtin_elementwise_min(__builtin_elementwise_max(v, (f16x2){(_Float16)0.0f, (_Float16)0.0f}),
                                         (f16x2){(_Float16)1.0f, (_Float16)1.0f});
    };
    const f16x2 t0 = clamp01(u0 * u0), t1 = clamp01(u1 * u1);
    f16x2 p0 = c(1.60618985f), p1 = c(1.60618985f);
    p0 = __builtin_elementwise_fma(p0, t0, c(-6.98037448f));
    p1 = __builtin_elementwise_fma(p1, t1, c(-6.98037448f));
    p0 = __builtin_elementwise_fma(p0, t0, c(12.9487521f));
    p1 = __builtin_elementwise_fma(p1, t1, c(12.9487521f));
    p0 = __builtin_elementwise_fma(p0, t0, c(-13.5802262f));
    p1 = __builtin_elementwise_fma(p1, t1, c(-13.5802262f));
    p0 = __builtin_elementwise_fma(p0, t0, c(9.05178404f));
    p1 = __builtin_elementwise_fma(p1, t1, c(9.05178404f));
    p0 = __builtin_elementwise_fma(p0, t0, c(-4.1370718f));
    p1 = __builtin_elementwise_fma(p1, t1, c(-4.1370718f));
    p0 = __builtin_elementwise_fma(p0, t0, c(1.59098072f));
    p1 = __builtin_elementwise_fma(p1, t1, c(1.59098072f));
    u0 = u0 * clamp01(__builtin_elementwise_fma(u0, p0, c(0.5f)));
    u1 = u1 * clamp01(__builtin_elementwise_fma(u1, p1, c(0.5f)));
}

__device__ __forceinline__ f16x2 to_f16x2(float a, float b) {
    return __builtin_bit_cast(f16x2, __builtin_amdgcn_cvt_pkrtz(a, b));
}

// Input feature (weight column) of k position p = 32 s + 8 g + j of a layer.
__device__ __forceinline__ int v2_column(int layer, int s, int g, int j) {
    if (layer == 0) {
        const int f = 16 * s + 4 * g + (j & 3);
        return j < 4 ? f : kFreq + f;
    }
    return j < 4 ? 32 * s + 4 * g + j : 32 * s + 16 + 4 * g + (j - 4);
}

// Fragment-major f16 copies of W1..W4 in the kernel's k order.
__global__ void v2_weights_kernel(const float* __restrict__ params, MlpLayout lay, _Float16* __restrict__ wfrag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one fragment lane (8 halves)
    const int64_t n1 = (int64_t)kL1Frags * 64, nl = (int64_t)kLFrags * 64;
    if (e >= n1 + 3 * nl) return;
    int layer;
    int64_t r;
    if (e < n1) {
        layer = 0;
        r = e;
    } else {
        layer = 1 + (int)((e - n1) / nl);
        r = (e - n1) % nl;
    }
    const int S = layer == 0 ? 4 : 8;
    const int lane = (int)(r % 64);
    const int frag = (int)(r / 64);
    const int mt = frag / S, s = frag % S;
    const int mrow = mt * 16 + (lane & 15), g = lane >> 4;
    const int K = lay.fan_in[layer];
    const float* W = params + lay.w_off[layer];
    // layer 1 is scaled by 1/4 (the kernel's accumulators hold z / 4); the inputs
    // of layers 2..4 arrive divided by 4, so their weights stay as they are
    const float sc = layer == 0 ? 0.25f : 1.0f;
    for (int j = 0; j < 8; ++j) wfrag[e * 8 + j] = (_Float16)(sc * W[(int64_t)mrow * K + v2_column(layer, s, g, j)]);
}

// Copies N fragments (N * 64 16-byte lanes), starting at byte `first` of the
// fragment buffer, into LDS with the block's 512 threads by buffer loads that
// write LDS directly: no registers are held and all of a thread's loads are in
// flight at once (the caller waits and synchronises).  The buffer descriptor's
// size bound makes any read past the fragments return zeros.
template <int N>
__device__ __forceinline__ void stage_frags(__amdgpu_buffer_rsrc_t rsrc, uint32_t first, _Float16* dst, int tid) {
    constexpr int kPer = N * 64 / 512;
    const int wave = tid >> 6;
    uint4* d = reinterpret_cast<uint4*>(dst) + wave * 64;  // lane l of the wave lands at d + l
#pragma unroll
    for (int k = 0; k < kPer; ++k)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void*)(d + k * 512), 16,
                                                 (uint32_t)tid * 16u, first + (uint32_t)k * 8192u, 0, 0);
}

__device__ __forceinline__ void stage_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Half h of layer L: output groups 4h..4h+3, i.e. fragments [h, h + 1) * (half
// of the layer's fragments); layer 1 has 32 fragments per half, the others 64.
template <int L, int H>
__device__ __forceinline__ void stage_half(__amdgpu_buffer_rsrc_t rsrc, _Float16* dst, int tid) {
    constexpr int kHalf = (L == 0 ? kL1Frags : kLFrags) / 2;
    constexpr uint32_t first = (uint32_t)((L == 0 ? 0 : kL1Frags + (L - 1) * kLFrags) + H * kHalf) * kFragHalves * 2;
    stage_frags<kHalf>(rsrc, first, dst, tid);
}

__global__ __launch_bounds__(512) void infer_v2_kernel(InferV2Args a) {
    // The weights of a layer in two 64 KB halves: wa holds output groups 0-3, wb
    // groups 4-7.  Each half is refilled with the next half as soon as every wave
    // is done with it, so a copy overlaps half a layer of MFMAs.
    __shared__ __attribute__((aligned(16))) _Float16 wa[kLFrags / 2 * kFragHalves];
    __shared__ __attribute__((aligned(16))) _Float16 wb[kLFrags / 2 * kFragHalves];
    __shared__ float bias_s[4][256];
    __shared__ float ff_s[kFreq * 5];
    // head weights (times 4) as row 0 of a 16-row A operand, one fragment per k-step
    __shared__ __attribute__((aligned(16))) _Float16 head_s[8 * kFragHalves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, nn = lane & 15;
    // Every layer computes u = z / 4 and passes on gelu(z) / 4 (powers of two, so
    // exact): biases are scaled by 1/4 here, layer 1's weights by 1/4 in the
    // fragment copy, and the head's weights by 4.
    for (int i = tid; i < 4 * 256; i += 512)
        bias_s[i / 256][i % 256] = 0.25f * a.params[a.lay.b_off[i / 256] + i % 256];
    for (int i = tid; i < kFreq * 5; i += 512) ff_s[i] = a.ff[i];
    for (int i = tid; i < 8 * 64; i += 512) {
        const int s = i >> 6, l = i & 63;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            head_s[i * 8 + j] =
                (l & 15) == 0 ? (_Float16)(4.0f * a.params[a.lay.w_off[4] + v2_column(1, s, l >> 4, j)]) : (_Float16)0.0f;
    }
    const float b5 = a.params[a.lay.b_off[4]];
    const __amdgpu_buffer_rsrc_t wrsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)a.wfrag, (short)0, (int)((kL1Frags + 3 * kLFrags) * kFragHalves * 2), 0x00020000);
    const int64_t cells = (int64_t)a.gnx * a.gny;
    // row -> (map, cell) by fp64 reciprocals: rows stay below 2^40, so the
    // quotient is off by at most one and a single correction makes it exact
    const double inv_cells = 1.0 / (double)cells, inv_gnx = 1.0 / (double)a.gnx;
    const int64_t step = (int64_t)gridDim.x * kV2Rows;
    if ((int64_t)blockIdx.x * kV2Rows < a.total) stage_half<0, 0>(wrsrc, wa, tid);
    for (int64_t base = (int64_t)blockIdx.x * kV2Rows; base < a.total; base += step) {
        int64_t row[2];
        float v[2][5];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            int64_t r = base + wave * 32 + t * 16 + nn;
            row[t] = r;
            if (r >= a.total) r = a.total - 1;
            int64_t ti = (int64_t)((double)r * inv_cells);
            int64_t c = r - ti * cells;
            if (c < 0) {
                --ti;
                c += cells;
            } else if (c >= cells) {
                ++ti;
                c -= cells;
            }
            int32_t iy = (int32_t)((double)c * inv_gnx);
            int32_t ix = (int32_t)c - iy * a.gnx;
            if (ix < 0) {
                --iy;
                ix += a.gnx;
            } else if (ix >= a.gnx) {
                ++iy;
                ix -= a.gnx;
            }
            v[t][0] = a.tx[3 * ti];
            v[t][1] = a.tx[3 * ti + 1];
            v[t][2] = a.tx[3 * ti + 2];
            v[t][3] = (float)(a.gx0 + (ix + 0.5) * a.gcell);
            v[t][4] = (float)(a.gy0 + (iy + 0.5) * a.gcell);
        }
        stage_wait();     // first half of layer 1 in wa
        __syncthreads();  // every wave done with wb (and the small tables are written)
        stage_half<0, 1>(wrsrc, wb, tid);
        // Fourier features as the first B operand: lane (g, nn), k-step s holds sin and
        // cos of frequencies 16 s + 4 g + 0..3 of its row
        f16x8 B[2][8];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            float vn[5];
#pragma unroll
            for (int i = 0; i < 5; ++i) vn[i] = (v[t][i] - a.norm.center[i]) * a.norm.inv_half[i];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                float sn[4], cs[4];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int f = 16 * s + 4 * g + jj;
                    float rev = 0.0f;
#pragma unroll
                    for (int i = 0; i < 5; ++i) rev = fmaf(ff_s[f * 5 + i], vn[i], rev);
                    sn[jj] = __builtin_amdgcn_sinf(rev);
                    cs[jj] = __builtin_amdgcn_cosf(rev);
                }
                const f16x2 h0 = to_f16x2(sn[0], sn[1]), h1 = to_f16x2(sn[2], sn[3]);
                const f16x2 h2 = to_f16x2(cs[0], cs[1]), h3 = to_f16x2(cs[2], cs[3]);
                B[t][s] = (f16x8){h0[0], h0[1], h1[0], h1[1], h2[0], h2[1], h3[0], h3[1]};
            }
        }
#pragma unroll
        for (int layer = 0; layer < 4; ++layer) {
            const int S = layer == 0 ? 4 : 8;
            if (layer > 0) {
                stage_wait();     // first half of this layer in wa
                __syncthreads();  // every wave done with wb
                if (layer == 1) stage_half<1, 1>(wrsrc, wb, tid);
                if (layer == 2) stage_half<2, 1>(wrsrc, wb, tid);
                if (layer == 3) stage_half<3, 1>(wrsrc, wb, tid);
            }
            // software pipeline over the 8 output groups (32 features each): the
            // GELU of group q - 1 is interleaved with the MFMAs of group q, one of
            // its four packed pairs per n-tile after each k-step
            f16x8 Bn[2][8];
            floatx4 accp[2][2];
            f16x2 hp[2][4];
#pragma unroll
            for (int q = 0; q <= 8; ++q) {
                if (q == 4) {
                    stage_wait();     // second half of this layer in wb
                    __syncthreads();  // every wave done with wa
                    if (layer == 0) stage_half<1, 0>(wrsrc, wa, tid);
                    if (layer == 1) stage_half<2, 0>(wrsrc, wa, tid);
                    if (layer == 2) stage_half<3, 0>(wrsrc, wa, tid);
                    if (layer == 3 && base + step < a.total) stage_half<0, 0>(wrsrc, wa, tid);  // next pass
                }
                floatx4 acc[2][2];
                if (q < 8) {
#pragma unroll
                    for (int mi = 0; mi < 2; ++mi) {
                        const int m0 = (2 * q + mi) * 16 + 4 * g;
                        const floatx4 b = {bias_s[layer][m0], bias_s[layer][m0 + 1], bias_s[layer][m0 + 2],
                                           bias_s[layer][m0 + 3]};
                        acc[mi][0] = b;
                        acc[mi][1] = b;
                    }
                }
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    if (q < 8 && s < S) {
                        const _Float16* w = q < 4 ? wa : wb;
                        const int qq = q & 3;
                        const f16x8 A0 =
                            *reinterpret_cast<const f16x8*>(w + ((2 * qq) * S + s) * kFragHalves + lane * 8);
                        const f16x8 A1 =
                            *reinterpret_cast<const f16x8*>(w + ((2 * qq + 1) * S + s) * kFragHalves + lane * 8);
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            acc[0][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A0, B[t][s], acc[0][t], 0, 0, 0);
                            acc[1][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1, B[t][s], acc[1][t], 0, 0, 0);
                        }
                    }
                    if (q > 0 && s < 4) {  // pair s of the previous group, both n-tiles
                        const int mi = s >> 1, r = (s & 1) * 2;
                        hp[0][s] = to_f16x2(accp[mi][0][r], accp[mi][0][r + 1]);
                        hp[1][s] = to_f16x2(accp[mi][1][r], accp[mi][1][r + 1]);
                        gelu2x2(hp[0][s], hp[1][s]);
                    }
                }
                if (q > 0) {
#pragma unroll
                    for (int t = 0; t < 2; ++t)
                        Bn[t][q - 1] = (f16x8){hp[t][0][0], hp[t][0][1], hp[t][1][0], hp[t][1][1],
                                               hp[t][2][0], hp[t][2][1], hp[t][3][0], hp[t][3][1]};
                }
                if (q < 8) {
#pragma unroll
                    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                        for (int t = 0; t < 2; ++t) accp[mi][t] = acc[mi][t];
                }
            }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int q = 0; q < 8; ++q) B[t][q] = Bn[t][q];
        }
        // head: output row 0 of C = W5 B lands in element 0 of the lanes with g = 0
        floatx4 hy[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const f16x8 A = *reinterpret_cast<const f16x8*>(head_s + s * kFragHalves + lane * 8);
#pragma unroll
            for (int t = 0; t < 2; ++t) hy[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, B[t][s], hy[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 2; ++t)
            if (g == 0 && row[t] < a.total)
                a.out[row[t]] = hy[t][0] + b5 + prior_db(a.norm, v[t][0], v[t][1], v[t][2], v[t][3], v[t][4]);
    }
}

// Number of nonzero bytes of a mask (atomic count).
__global__ void count_u8_kernel(const uint8_t* __restrict__ m, int64_t n, unsigned long long* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool on = i < n && m[i] != 0;
    const uint64_t b = __ballot(on);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (unsigned long long)__popcll(b));
}

// Traced cells replace predicted ones: out[c] = 10 log10(gain[c]) (-inf when
// no ray crossed the cell) where fallback[c] != 0.
__global__ void fallback_merge_kernel(const uint8_t* __restrict__ fallback, const float* __restrict__ gain,
                                      int64_t n, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !fallback[i]) return;
    const float g = gain[i];
    out[i] = g > 0.0f ? 10.0f * log10f(g) : -__builtin_inff();
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

hipError_t launch_rowsum(const bf16* dZt, int64_t rows, int64_t cols, float* db, hipStream_t s) {
    hipLaunchKernelGGL(rowsum_kernel, dim3((unsigned)rows), dim3(256), 0, s, dZt, cols, db);
    return hipGetLastError();
}

hipError_t launch_reduce_splits(const float* part, int S, int64_t n, float* grad, hipStream_t s) {
    hipLaunchKernelGGL(reduce_splits_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, part, S, n, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_init(float* params, float* ff, uint64_t seed, const MlpFourier& fs, const MlpLayout& lay,
                           hipStream_t s) {
    hipLaunchKernelGGL(init_kernel, dim3(blocks_for(lay.total, 256)), dim3(256), 0, s, params, ff, seed, fs, lay);
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

int64_t v2_weights_halves() { return (int64_t)(kL1Frags + 3 * kLFrags) * kFragHalves; }

hipError_t launch_count_u8(const uint8_t* m, int64_t n, unsigned long long* count, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(count_u8_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, m, n, count);
    return hipGetLastError();
}

hipError_t launch_fallback_merge(const uint8_t* fallback, const float* gain, int64_t n, float* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fallback_merge_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, fallback, gain, n, out);
    return hipGetLastError();
}

hipError_t launch_infer_v2(const float* tx, int32_t T, double gx0, double gy0, double gcell, int32_t gnx, int32_t gny,
                           const float* ff, const MlpNorm& norm, _Float16* wfrag, const MlpLayout& lay,
                           const float* params, float* out, int grid, hipStream_t s) {
    const int64_t lanes = (int64_t)(kL1Frags + 3 * kLFrags) * 64;
    hipLaunchKernelGGL(v2_weights_kernel, dim3(blocks_for(lanes, 256)), dim3(256), 0, s, params, lay, wfrag);
    InferV2Args a;
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
    a.wfrag = wfrag;
    a.params = params;
    a.lay = lay;
    a.out = out;
    const int64_t passes = (a.total + kV2Rows - 1) / kV2Rows;
    const unsigned blocks = (unsigned)std::min<int64_t>(passes, grid);
    hipLaunchKernelGGL(infer_v2_kernel, dim3(blocks), dim3(512), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_map_inputs(const float* tx, int32_t T, double gx0, double gy0, double gcell, int32_t gnx,
                             int32_t gny, int64_t row0, int64_t rows, float* v, hipStream_t s) {
    hipLaunchKernelGGL(map_inputs_kernel, dim3(blocks_for(rows, 256)), dim3(256), 0, s, tx, T, gx0, gy0, gcell, gnx,
                       gny, row0, rows, v);
    return hipGetLastError();
}

}  // namespace rt
