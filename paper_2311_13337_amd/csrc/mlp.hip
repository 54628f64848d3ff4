// mlp.hip -- surrogate network 4 -> 128 -> 128 -> 6 (GELU) on CDNA4.
//
// Matrix products take bfloat16 operands (round to nearest even) and
// accumulate in FP32: the 128 x 128 products on MFMA (v_mfma_f32_16x16x16
// bf16), the 4-wide and 6-wide ones on the vector ALU (a product of two
// bfloat16 values is exact in FP32, so only the summation order differs from
// MFMA). Biases, GELU (exact erf form), losses and Adam run in FP32.
//
//  mlp_grad_kernel    one workgroup per tile of 32 samples: forward, MSE
//                     gradient, backward; writes the tile's parameter gradient
//                     and loss to a per-tile slot (no atomics)
//  mlp_adam_kernel    sums the tile slots in fixed order and applies Adam
//  mlp_predict_kernel forward pass, de-normalised outputs, and optionally the
//                     Jacobian dY_n/dx_n by forward-mode tangents
#include <hip/hip_runtime.h>
#include <math.h>

#include "mlp_engine.h"

namespace vadx {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float rbf(float x) { return from_bf16(to_bf16(x)); }

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x)
{
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
           x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// One 16x16 output tile of C += A B with K a multiple of 16, A and B bf16 in
// LDS, addressed through strides: A[i][k] = a[i * a_rs + k * a_cs], B[k][j] =
// b[k * b_rs + j * b_cs]. Lane l holds A[l%16][4(l/16)..+3], B[4(l/16)..+3][l%16]
// and returns C[4(l/16)..+3][l%16].
__device__ __forceinline__ f32x4 mfma_tile(const uint16_t *a, int a_rs, int a_cs, const uint16_t *b,
                                           int b_rs, int b_cs, int K, f32x4 acc)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, kg = lane >> 4;
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 av, bv;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = k0 + 4 * kg + t;
            av[t] = (short)a[r * a_rs + k * a_cs];
            bv[t] = (short)b[k * b_rs + r * b_cs];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
    return acc;
}

constexpr int T = kMlpTile;   // samples per workgroup
constexpr int H = 128;

constexpr int kStageBatch = 16;   // W2 loads in flight per thread (H * H = 4 batches of 256 x 16)
static_assert((H * H) % (kStageBatch * 256) == 0, "W2 staging covers whole batches");

// W2 to bfloat16 in LDS by a 256-thread workgroup, kStageBatch loads in flight
// per thread before their conversions (one load and wait at a time, the staging
// was most of a gradient launch).
__device__ inline void stage_w2(uint16_t *W2b, const float *W2, int tid)
{
    for (int i0 = tid; i0 < H * H; i0 += kStageBatch * 256) {
        float v[kStageBatch];
#pragma unroll
        for (int j = 0; j < kStageBatch; ++j) v[j] = W2[i0 + j * 256];
#pragma unroll
        for (int j = 0; j < kStageBatch; ++j) W2b[i0 + j * 256] = to_bf16(v[j]);
    }
}

__global__ __launch_bounds__(256) void mlp_grad_kernel(MlpArgs a, const float *__restrict__ X,
                                                       const float *__restrict__ Y, int n,
                                                       float inv_n6)
{
    __shared__ uint16_t W2b[H * H];          // W2 [n_out][k] bf16
    __shared__ uint16_t H1b[T * H], H2b[T * H], dZ2b[T * H];
    __shared__ float Z1[T * H], Z2[T * H];
    __shared__ float W1s[H * 4], W3s[6 * H], Xs[T * 4], Ys[T * 6], dYs[T * 6];
    __shared__ float red[256];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int s0 = blockIdx.x * T;
    const float *W1 = a.params, *b1 = W1 + H * 4, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H,
                *b3 = W3 + 6 * H;
    float *g = a.partial + (int64_t)blockIdx.x * kMlpSlot;
    stage_w2(W2b, W2, tid);
    for (int i = tid; i < H * 4; i += 256) W1s[i] = rbf(W1[i]);
    for (int i = tid; i < 6 * H; i += 256) W3s[i] = rbf(W3[i]);
    for (int i = tid; i < T * 4; i += 256) {
        const int s = i >> 2, c = i & 3;
        float x = 0.f;
        if (s0 + s < n) x = (X[(int64_t)(s0 + s) * 4 + c] - a.x_lo[c]) * a.x_scale[c] - 1.0f;
        Xs[i] = rbf(x);
    }
    for (int i = tid; i < T * 6; i += 256) {
        const int s = i / 6, c = i - s * 6;
        Ys[i] = (s0 + s < n) ? (Y[(int64_t)(s0 + s) * 6 + c] - a.y_mean[c]) * a.y_rstd[c] : 0.f;
    }
    __syncthreads();
    // layer 1 (vector ALU): Z1 = X W1^T + b1
    for (int i = tid; i < T * H; i += 256) {
        const int s = i >> 7, j = i & (H - 1);
        float z = b1[j];
#pragma unroll
        for (int c = 0; c < 4; ++c) z = fmaf(Xs[s * 4 + c], W1s[j * 4 + c], z);
        Z1[i] = z;
        H1b[i] = to_bf16(gelu(z));
    }
    __syncthreads();
    // layer 2 (MFMA): Z2 = H1 W2^T + b2; 2 x 8 output tiles over 4 waves
    for (int t = wave; t < (T / 16) * (H / 16); t += 4) {
        const int ti = t / (H / 16), tj = t % (H / 16);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma_tile(H1b + ti * 16 * H, H, 1, W2b + tj * 16 * H, 1, H, H, acc);
        const int j = tj * 16 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int s = ti * 16 + 4 * (lane >> 4) + q;
            const float z = acc[q] + b2[j];
            Z2[s * H + j] = z;
            H2b[s * H + j] = to_bf16(gelu(z));
        }
    }
    __syncthreads();
    // layer 3 (vector ALU) and the loss gradient
    float lsum = 0.f;
    for (int i = tid; i < T * 6; i += 256) {
        const int s = i / 6, o = i - s * 6;
        float y = b3[o];
        for (int k = 0; k < H; ++k) y = fmaf(from_bf16(H2b[s * H + k]), W3s[o * H + k], y);
        const float d = (s0 + s < n) ? y - Ys[i] : 0.f;
        lsum = fmaf(d, d, lsum);
        dYs[i] = 2.0f * d * inv_n6;
    }
    red[tid] = lsum;
    __syncthreads();
    // dW3 = dY^T H2, db3 = sum dY
    for (int i = tid; i < 6 * H; i += 256) {
        const int o = i >> 7, k = i & (H - 1);
        float acc = 0.f;
        for (int s = 0; s < T; ++s) acc = fmaf(rbf(dYs[s * 6 + o]), from_bf16(H2b[s * H + k]), acc);
        g[kMlpOffW3 + i] = acc;
    }
    if (tid < 6) {
        float acc = 0.f;
        for (int s = 0; s < T; ++s) acc += dYs[s * 6 + tid];
        g[kMlpOffB3 + tid] = acc;
    }
    if (tid == 0) {
        float l = 0.f;
        for (int i = 0; i < 256; ++i) l += red[i];
        g[kMlpOffLoss] = l;
    }
    // dH2 = dY W3, dZ2 = dH2 * gelu'(Z2)
    for (int i = tid; i < T * H; i += 256) {
        const int s = i >> 7, k = i & (H - 1);
        float acc = 0.f;
#pragma unroll
        for (int o = 0; o < 6; ++o) acc = fmaf(rbf(dYs[s * 6 + o]), W3s[o * H + k], acc);
        const float dz = acc * gelu_grad(Z2[i]);
        Z2[i] = dz;                       // Z2 now holds dZ2 (FP32) for db2
        dZ2b[i] = to_bf16(dz);
    }
    __syncthreads();
    // db2 = sum_s dZ2
    for (int j = tid; j < H; j += 256) {
        float acc = 0.f;
        for (int s = 0; s < T; ++s) acc += Z2[s * H + j];
        g[kMlpOffB2 + j] = acc;
    }
    // dW2 = dZ2^T H1 (MFMA, K = T samples): 8 x 8 tiles over 4 waves
    for (int t = wave; t < (H / 16) * (H / 16); t += 4) {
        const int ti = t / (H / 16), tj = t % (H / 16);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        // A[i][k] = dZ2[k][ti*16+i], B[k][j] = H1[k][tj*16+j]
        acc = mfma_tile(dZ2b + ti * 16, 1, H, H1b + tj * 16, H, 1, T, acc);
        const int j = tj * 16 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = ti * 16 + 4 * (lane >> 4) + q;
            g[kMlpOffW2 + i * H + j] = acc[q];
        }
    }
    // dH1 = dZ2 W2 (MFMA, K = 128): A[s][k] = dZ2[s][k], B[k][j] = W2[k][j]
    for (int t = wave; t < (T / 16) * (H / 16); t += 4) {
        const int ti = t / (H / 16), tj = t % (H / 16);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma_tile(dZ2b + ti * 16 * H, H, 1, W2b + tj * 16, H, 1, H, acc);
        const int j = tj * 16 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int s = ti * 16 + 4 * (lane >> 4) + q;
            Z1[s * H + j] = acc[q] * gelu_grad(Z1[s * H + j]);   // Z1 now holds dZ1
        }
    }
    __syncthreads();
    // dW1 = dZ1^T X, db1 = sum dZ1
    for (int i = tid; i < H * 4; i += 256) {
        const int j = i >> 2, c = i & 3;
        float acc = 0.f;
        for (int s = 0; s < T; ++s) acc = fmaf(rbf(Z1[s * H + j]), Xs[s * 4 + c], acc);
        g[kMlpOffW1 + i] = acc;
    }
    for (int j = tid; j < H; j += 256) {
        float acc = 0.f;
        for (int s = 0; s < T; ++s) acc += Z1[s * H + j];
        g[kMlpOffB1 + j] = acc;
    }
}

// Sums slot entry e of the n_tiles tile slots in tile order, kSumBatch loads
// in flight at a time.
constexpr int kSumBatch = 8;
__device__ inline float tile_sum(const float *partial, int n_tiles, int e)
{
    float gs = 0.f;
    int t = 0;
    for (; t + kSumBatch <= n_tiles; t += kSumBatch) {
        float v[kSumBatch];
#pragma unroll
        for (int u = 0; u < kSumBatch; ++u) v[u] = partial[(int64_t)(t + u) * kMlpSlot + e];
#pragma unroll
        for (int u = 0; u < kSumBatch; ++u) gs += v[u];
    }
    for (; t < n_tiles; ++t) gs += partial[(int64_t)t * kMlpSlot + e];
    return gs;
}

// Sums the tile gradients in tile order (deterministic) and applies Adam.
// c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t). apply = 0 only sums (gradient
// read-out); the loss sum goes to a.loss_out[step], taken by the thread past
// the last parameter (the grid holds one) alongside the parameters' sums.
__global__ void mlp_adam_kernel(MlpArgs a, int n_tiles, float c1, float c2, int apply, int step)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) {
        const float gs = tile_sum(a.partial, n_tiles, p);
        a.grad[p] = gs;
        if (apply) {
            const float m = a.beta1 * a.m[p] + (1.f - a.beta1) * gs;
            const float v = a.beta2 * a.v[p] + (1.f - a.beta2) * gs * gs;
            a.m[p] = m;
            a.v[p] = v;
            a.params[p] -= a.lr * (m * c1) / (sqrtf(v * c2) + a.eps);
        }
    }
    if (p == kMlpParams && a.loss_out) a.loss_out[step] = tile_sum(a.partial, n_tiles, kMlpOffLoss);
}

// Forward pass for tiles of 32 points; Jacobian by forward-mode tangents:
// T1 = g1' W1 (per sample 128 x 4), T2 = g2' (W2 T1), J = W3 T2. Each 16 x 16
// tile of T2 is folded into J at once (LDS float atomics), so T2 is never
// stored. score (optional) = |dY_o0/dx_n|^2 + |dY_o1/dx_n|^2 per point.
__global__ __launch_bounds__(256) void mlp_predict_kernel(MlpArgs a, const float *__restrict__ X,
                                                          int64_t n, float *__restrict__ Yout,
                                                          float *__restrict__ Jout,
                                                          float *__restrict__ score)
{
    __shared__ uint16_t W2b[H * H];
    __shared__ uint16_t H1b[T * H];
    __shared__ uint16_t T1b[T * 4 * H];      // rows (s, input c), 128 columns
    __shared__ float G2[T * H];
    __shared__ float H2s[T * H];
    __shared__ float W1s[H * 4], W3s[6 * H], Xs[T * 4];
    __shared__ float Jacc[T * 4 * 6];        // [s][c][o]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t s0 = (int64_t)blockIdx.x * T;
    const bool jac = Jout != nullptr || score != nullptr;
    const float *W1 = a.params, *b1 = W1 + H * 4, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H,
                *b3 = W3 + 6 * H;
    stage_w2(W2b, W2, tid);
    for (int i = tid; i < H * 4; i += 256) W1s[i] = rbf(W1[i]);
    for (int i = tid; i < 6 * H; i += 256) W3s[i] = rbf(W3[i]);
    for (int i = tid; i < T * 4 * 6; i += 256) Jacc[i] = 0.f;
    for (int i = tid; i < T * 4; i += 256) {
        const int s = i >> 2, c = i & 3;
        float x = 0.f;
        if (s0 + s < n) x = (X[(s0 + s) * 4 + c] - a.x_lo[c]) * a.x_scale[c] - 1.0f;
        Xs[i] = rbf(x);
    }
    __syncthreads();
    for (int i = tid; i < T * H; i += 256) {
        const int s = i >> 7, j = i & (H - 1);
        float z = b1[j];
#pragma unroll
        for (int c = 0; c < 4; ++c) z = fmaf(Xs[s * 4 + c], W1s[j * 4 + c], z);
        H1b[i] = to_bf16(gelu(z));
        if (jac) {
            const float g1 = gelu_grad(z);
#pragma unroll
            for (int c = 0; c < 4; ++c) T1b[(s * 4 + c) * H + j] = to_bf16(g1 * W1s[j * 4 + c]);
        }
    }
    __syncthreads();
    for (int t = wave; t < (T / 16) * (H / 16); t += 4) {
        const int ti = t / (H / 16), tj = t % (H / 16);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma_tile(H1b + ti * 16 * H, H, 1, W2b + tj * 16 * H, 1, H, H, acc);
        const int j = tj * 16 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int s = ti * 16 + 4 * (lane >> 4) + q;
            const float z = acc[q] + b2[j];
            H2s[s * H + j] = rbf(gelu(z));
            G2[s * H + j] = gelu_grad(z);
        }
    }
    __syncthreads();
    if (jac) {
        for (int t = wave; t < (T * 4 / 16) * (H / 16); t += 4) {
            const int ti = t / (H / 16), tj = t % (H / 16);
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma_tile(T1b + ti * 16 * H, H, 1, W2b + tj * 16 * H, 1, H, H, acc);
            const int j = tj * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = ti * 16 + 4 * (lane >> 4) + q;   // row = s * 4 + c
                const float t2 = rbf(acc[q] * G2[(row >> 2) * H + j]);
#pragma unroll
                for (int o = 0; o < 6; ++o) atomicAdd(&Jacc[row * 6 + o], W3s[o * H + j] * t2);
            }
        }
        __syncthreads();
    }
    // outputs: Y = H2 W3^T + b3 (de-normalised); J in normalised units
    for (int i = tid; i < T * 6; i += 256) {
        const int s = i / 6, o = i - s * 6;
        if (s0 + s >= n) continue;
        float y = b3[o];
        for (int k = 0; k < H; ++k) y = fmaf(H2s[s * H + k], W3s[o * H + k], y);
        Yout[(s0 + s) * 6 + o] = y * a.y_std[o] + a.y_mean[o];
        if (Jout)
#pragma unroll
            for (int c = 0; c < 4; ++c) Jout[((s0 + s) * 6 + o) * 4 + c] = Jacc[(s * 4 + c) * 6 + o];
    }
    if (score)
        for (int s = tid; s < T; s += 256) {
            if (s0 + s >= n) continue;
            float ss = 0.f;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float u = Jacc[(s * 4 + c) * 6 + a.score_out0];
                const float w = Jacc[(s * 4 + c) * 6 + a.score_out1];
                ss = fmaf(u, u, fmaf(w, w, ss));
            }
            score[s0 + s] = sqrtf(ss);
        }
}

hipError_t launch_mlp_grad(const MlpArgs &a, const float *X, const float *Y, int n, int n_total,
                           hipStream_t s)
{
    const int tiles = (n + T - 1) / T;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(tiles), dim3(256), 0, s, a, X, Y, n,
                       1.0f / (6.0f * (float)n_total));
    return hipGetLastError();
}

hipError_t launch_mlp_adam(const MlpArgs &a, int n_tiles, float c1, float c2, int apply, int step,
                           hipStream_t s)
{
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, s, a,
                       n_tiles, c1, c2, apply, step);
    return hipGetLastError();
}

hipError_t launch_mlp_predict(const MlpArgs &a, const float *X, int64_t n, float *Y, float *J,
                              float *score, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t tiles = (n + T - 1) / T;
    hipLaunchKernelGGL(mlp_predict_kernel, dim3((unsigned)tiles), dim3(256), 0, s, a, X, n, Y, J,
                       score);
    return hipGetLastError();
}

} // namespace vadx
