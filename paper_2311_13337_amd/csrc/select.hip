// select.hip -- selection of the points to simulate after screening a grid
// with the surrogate: the k points of largest score (ties broken towards the
// lower index) plus an audit sample of the others, each independently with a
// given probability from a Philox draw keyed by the point index.
//
// Top-k uses a radix select on order-preserving 32-bit keys (four 8-bit
// histogram passes find the k-th largest key T exactly), then a three-phase
// stream compaction in index order: per-tile counts of keys equal to T, per-
// tile counts of selected points, and the write. Tiles are 4096 consecutive
// points (256 threads x 16); the two small exclusive scans over tiles run on
// the host between phases.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_engine.h"
#include "philox.h"

namespace vadx {

constexpr int kSelThreads = 256;
constexpr int kSelPer = 16;

__device__ __forceinline__ uint32_t order_key(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ bool audit_draw(uint32_t seed, int64_t i, float frac)
{
    uint32_t c[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u, 0u};
    philox4x32_10(c, seed, 0xA0D17u);
    return (float)(c[0] >> 8) * 5.9604644775390625e-08f < frac;   // 2^-24
}

__global__ __launch_bounds__(kSelThreads) void sel_hist_kernel(const float *__restrict__ score,
                                                              int64_t n, uint32_t prefix,
                                                              uint32_t mask, int shift,
                                                              uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kSelThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kSelThreads) {
        const uint32_t k = order_key(score[i]);
        if ((k & mask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Exclusive scan of one value per thread over the workgroup; returns the
// thread's exclusive prefix and writes the total to *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *buf, uint32_t *total)
{
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < kSelThreads; off <<= 1) {
        const uint32_t add = t >= off ? buf[t - off] : 0u;
        __syncthreads();
        buf[t] += add;
        __syncthreads();
    }
    const uint32_t incl = buf[t];
    *total = buf[kSelThreads - 1];
    __syncthreads();
    return incl - v;
}

// phase 0: out[tile] = number of keys == T in the tile
// phase 1: out[tile] = number of selected points in the tile (needs eq_base)
// phase 2: writes the selected indices at sel_base[tile] + rank (needs both)
__global__ __launch_bounds__(kSelThreads) void sel_compact_kernel(
    const float *__restrict__ score, int64_t n, int phase, int use_top, uint32_t T, int64_t need,
    float audit_frac, uint32_t seed, const int64_t *__restrict__ eq_base,
    const int64_t *__restrict__ sel_base, uint32_t *__restrict__ out, int64_t *__restrict__ sel,
    uint8_t *__restrict__ is_audit)
{
    __shared__ uint32_t buf[kSelThreads];
    const int64_t i0 = (int64_t)blockIdx.x * (kSelThreads * kSelPer) + (int64_t)threadIdx.x * kSelPer;
    uint32_t keys[kSelPer];
    uint32_t n_eq = 0;
#pragma unroll
    for (int q = 0; q < kSelPer; ++q) {
        keys[q] = (i0 + q < n) ? order_key(score[i0 + q]) : 0u;
        n_eq += (use_top && i0 + q < n && keys[q] == T) ? 1u : 0u;
    }
    uint32_t tot;
    if (phase == 0) {
        block_exclusive_scan(n_eq, buf, &tot);
        if (threadIdx.x == 0) out[blockIdx.x] = tot;
        return;
    }
    int64_t eq_rank = eq_base[blockIdx.x] + block_exclusive_scan(n_eq, buf, &tot);
    uint32_t picked = 0;   // bit q: point i0 + q selected
    uint32_t audit = 0;
#pragma unroll
    for (int q = 0; q < kSelPer; ++q) {
        if (i0 + q >= n) continue;
        bool top = false;
        if (use_top) {
            if (keys[q] > T) {
                top = true;
            } else if (keys[q] == T) {
                top = eq_rank < need;
                ++eq_rank;
            }
        }
        const bool aud = !top && audit_frac > 0.f && audit_draw(seed, i0 + q, audit_frac);
        if (top || aud) picked |= 1u << q;
        if (aud) audit |= 1u << q;
    }
    const uint32_t cnt = __popc(picked);
    const uint32_t rank = block_exclusive_scan(cnt, buf, &tot);
    if (phase == 1) {
        if (threadIdx.x == 0) out[blockIdx.x] = tot;
        return;
    }
    int64_t w = sel_base[blockIdx.x] + rank;
#pragma unroll
    for (int q = 0; q < kSelPer; ++q)
        if (picked & (1u << q)) {
            sel[w] = i0 + q;
            if (is_audit) is_audit[w] = (audit >> q) & 1u;
            ++w;
        }
}

int64_t select_tiles(int64_t n) { return (n + kSelThreads * kSelPer - 1) / (kSelThreads * kSelPer); }

hipError_t launch_sel_hist(const float *score, int64_t n, uint32_t prefix, uint32_t mask, int shift,
                           uint32_t *hist, hipStream_t s)
{
    int64_t blocks = (n + kSelThreads - 1) / kSelThreads;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(sel_hist_kernel, dim3((unsigned)blocks), dim3(kSelThreads), 0, s, score, n,
                       prefix, mask, shift, hist);
    return hipGetLastError();
}

hipError_t launch_sel_compact(const float *score, int64_t n, int phase, int use_top, uint32_t T,
                              int64_t need, float audit_frac, uint32_t seed, const int64_t *eq_base,
                              const int64_t *sel_base, uint32_t *out, int64_t *sel,
                              uint8_t *is_audit, hipStream_t s)
{
    const int64_t tiles = select_tiles(n);
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(sel_compact_kernel, dim3((unsigned)tiles), dim3(kSelThreads), 0, s, score, n,
                       phase, use_top, T, need, audit_frac, seed, eq_base, sel_base, out, sel,
                       is_audit);
    return hipGetLastError();
}

} // namespace vadx
