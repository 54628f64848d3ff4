// kernels.hip -- HIP kernels of the TVB-AdEx sweep engine for CDNA4 (gfx950).
//
//  conn_prepare  row normalisation of the connectome weights and CSR build
//  delays        per (delay table, edge): round-half-even(L / (v dt)), >= 1
//  integrate     stochastic Heun of many networks: one lane per
//                (instance, region), instances of a workgroup share a region
//                count; coupling gathered from per-instance delay rings once per
//                block of B <= d_min + 1 steps; Philox noise in registers
//  fc_stats      Pearson FC (FP64 Gram of the rate samples) and statistics
#include <hip/hip_runtime.h>
#include <math.h>

#include "engine.h"

namespace vadx {

// ------------------------------------------------------------------ setup
__global__ void conn_prepare_kernel(int n, const double *__restrict__ w,
                                    const double *__restrict__ len, int32_t *__restrict__ rowptr,
                                    float *__restrict__ weight, double *__restrict__ edge_len,
                                    int32_t *__restrict__ colidx)
{
    __shared__ int32_t cnt[1025];
    const int k = threadIdx.x;
    double s = 0.0;
    int c = 0;
    if (k < n) {
        for (int j = 0; j < n; ++j) {
            double x = w[(int64_t)k * n + j];
            s += x;
            c += (x != 0.0);
        }
        cnt[k + 1] = c;
    }
    if (k == 0) cnt[0] = 0;
    __syncthreads();
    if (k == 0)
        for (int i = 1; i <= n; ++i) cnt[i] += cnt[i - 1];
    __syncthreads();
    if (k < n) {
        int e = cnt[k];
        rowptr[k] = e;
        if (k == n - 1) rowptr[n] = cnt[n];
        for (int j = 0; j < n; ++j) {
            double x = w[(int64_t)k * n + j];
            if (x != 0.0) {
                weight[e] = (float)(x / s);
                edge_len[e] = len[(int64_t)k * n + j];
                colidx[e] = j;
                ++e;
            }
        }
    }
}

hipError_t launch_conn_prepare(int n, const double *w, const double *len, int32_t *rowptr,
                               float *weight, double *edge_len, int32_t *colidx, hipStream_t s)
{
    int threads = ((n + 63) / 64) * 64;
    hipLaunchKernelGGL(conn_prepare_kernel, dim3(1), dim3(threads), 0, s, n, w, len, rowptr,
                       weight, edge_len, colidx);
    return hipGetLastError();
}

__global__ void delays_kernel(const DelayTableDev *__restrict__ tables,
                              const ConnDev *__restrict__ conns, const int32_t *__restrict__ colidx,
                              const double *__restrict__ edge_len, double dt,
                              int32_t *__restrict__ packed)
{
    const DelayTableDev t = tables[blockIdx.y];
    const ConnDev c = conns[t.conn];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < c.nnz; e += gridDim.x * blockDim.x) {
        double q = rint(edge_len[c.edge_off + e] / ((double)t.v * dt));
        int32_t d = q < 1.0 ? 1 : (int32_t)q;
        packed[t.off + e] = (colidx[c.edge_off + e] << 20) | d;
    }
}

hipError_t launch_delays(int n_tables, const DelayTableDev *tables, const ConnDev *conns,
                         const int32_t *colidx, const double *edge_len, double dt,
                         int32_t *packed, int max_nnz, hipStream_t s)
{
    if (n_tables == 0) return hipSuccess;
    int bx = (max_nnz + 255) / 256;
    if (bx > 64) bx = 64;
    if (bx < 1) bx = 1;
    hipLaunchKernelGGL(delays_kernel, dim3(bx, n_tables), dim3(256), 0, s, tables, conns,
                       colidx, edge_len, dt, packed);
    return hipGetLastError();
}

// ------------------------------------------------------------------ noise
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 products
// with the round keys bumped by the Weyl constants.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Four standard normals for steps 4q .. 4q+3 of region k: words mapped to
// (0, 1) as (w + 1/2) 2^-32, two Box-Muller (cos, sin) pairs.
__device__ __forceinline__ void normals4(uint32_t seed, uint32_t id, uint32_t q, uint32_t k,
                                         float z[4])
{
    uint32_t c[4] = {q, k, 0u, 0u};
    philox4x32_10(c, seed, id);
    const float s32 = 2.3283064365386963e-10f, h32 = 1.1641532182693481e-10f;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        float u0 = fmaf((float)c[2 * p], s32, h32);
        float u1 = fmaf((float)c[2 * p + 1], s32, h32);
        float rr = sqrtf(-2.0f * logf(u0));
        float sn, cs;
        sincospif(2.0f * u1, &sn, &cs);
        z[2 * p] = rr * cs;
        z[2 * p + 1] = rr * sn;
    }
}

// ------------------------------------------------------------------ integrate
template <int B>
__global__ __launch_bounds__(512) void integrate_kernel(IntegrateArgs a)
{
    extern __shared__ float cbuf[];   // [B][blockDim.x] coupling of the block's steps
    const GroupDev g = a.groups[blockIdx.x];
    const int tid = threadIdx.x;
    const int slot = tid / g.n;
    const int k = tid - slot * g.n;
    const bool active = slot < g.count;
    const int nthr = blockDim.x;

    InstDev I;
    ConnDev C;
    double X[8];
    float acc = 0.f;
    int row_b = 0, row_e = 0;
    const float *wrow = nullptr;
    const int32_t *prow = nullptr;
    float *ring = nullptr;
    float *trace = nullptr;
    int64_t tc = 0, sidx = 0;
    uint32_t fl = 0;
    if (active) {
        I = a.inst[a.perm[g.first + slot]];
        C = a.conns[I.conn];
        row_b = a.rowptr[C.row_off + k];
        row_e = a.rowptr[C.row_off + k + 1];
        wrow = a.weight + C.edge_off;
        prow = a.packed + I.table_off;
        ring = a.ws + I.ring_off;
        if (I.trace_off >= 0) trace = a.ws + I.trace_off;
        tc = a.n_begin % a.tavg_steps;
        sidx = a.n_begin / a.tavg_steps - a.transient_steps / a.tavg_steps;
        if (a.n_begin == 0) {
            X[0] = a.E_init;
            X[1] = a.I_init;
#pragma unroll
            for (int q = 2; q < 8; ++q) X[q] = 0.0;
            float *rr = ring + (int64_t)k * I.D;
            const float e0 = (float)a.E_init;
            for (int s = 0; s < I.D; ++s) rr[s] = e0;
        } else {
            const double *st = reinterpret_cast<const double *>(a.ws + I.state_off);
#pragma unroll
            for (int q = 0; q < 8; ++q) X[q] = st[q * I.n + k];
            acc = a.ws[I.acc_off + k];
        }
    }
    __syncthreads();   // initial rings visible to all lanes

    const float S = active ? I.S : 0.f, be = active ? I.be : 0.f, ae = active ? I.ae : 0.f;
    const int D = active ? I.D : 1;
    int nm = active ? (int)(a.n_begin % D) : 0;   // n0 mod D
    float z4[4] = {0.f, 0.f, 0.f, 0.f};

    for (int64_t n0 = a.n_begin; n0 < a.n_end; n0 += B) {
        const int nb = (int)((a.n_end - n0) < B ? (a.n_end - n0) : B);
        if (active) {
            // coupling of steps n0 .. n0+nb-1: S sum_j W_kj H_j[n - d_kj]
            float cb[B];
#pragma unroll
            for (int b = 0; b < B; ++b) cb[b] = 0.f;
            for (int e = row_b; e < row_e; ++e) {
                const int32_t pk = prow[e];
                const int j = pk >> 20, d = pk & 0xFFFFF;
                const float w = wrow[e];
                const float *hr = ring + (int64_t)j * D;
                int s0 = nm - d;
                s0 += (s0 < 0) ? D : 0;
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    if (b < nb) {
                        int sl = s0 + b;
                        sl -= (sl >= D) ? D : 0;
                        cb[b] = fmaf(w, hr[sl], cb[b]);
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < B; ++b) cbuf[b * nthr + tid] = S * cb[b];

            float *myrow = ring + (int64_t)k * D;
            int wm = nm;
            for (int b = 0; b < nb; ++b) {
                const int64_t n = n0 + b;
                const int r = (int)(n & 3);
                if (r == 0 || b == 0)
                    normals4(a.seed, I.id, (uint32_t)(n >> 2), (uint32_t)k, z4);
                const float z = r == 0 ? z4[0] : (r == 1 ? z4[1] : (r == 2 ? z4[2] : z4[3]));
                const float c = cbuf[b * nthr + tid];
                bool hit = step_region(a.M, a.integrator, a.dt, X, c, be, ae,
                                       a.gdw_scale * (double)z);
                double chk = ((X[0] + X[1]) + (X[2] + X[3])) + ((X[4] + X[5]) + (X[6] + X[7]));
                fl |= hit ? 2u : 0u;
                fl |= __builtin_isfinite(chk) ? 0u : 1u;
                // history of E: slot (n + 1) mod D
                wm += 1;
                wm -= (wm >= D) ? D : 0;
                const float e1 = (float)X[0];
                myrow[wm] = e1;
                // time average
                acc += e1;
                tc += 1;
                if (tc == a.tavg_steps) {
                    if (sidx >= 0 && sidx < a.n_samples)
                        a.ws[I.samp_off + sidx * I.n + k] = acc / (float)a.tavg_steps;
                    acc = 0.f;
                    tc = 0;
                    ++sidx;
                }
                if (trace != nullptr && n < a.n_trace_steps) {
                    float *tr = trace + n * 8 * I.n + k;
#pragma unroll
                    for (int q = 0; q < 8; ++q) tr[q * I.n] = (float)X[q];
                }
            }
            nm += nb;
            nm -= (nm >= D) ? D : 0;
        }
        __syncthreads();   // this block's history visible before the next block reads it
    }
    if (active) {
        double *st = reinterpret_cast<double *>(a.ws + I.state_off);
#pragma unroll
        for (int q = 0; q < 8; ++q) st[q * I.n + k] = X[q];
        a.ws[I.acc_off + k] = acc;
        if (fl) atomicOr(&a.flags[a.perm[g.first + slot]], fl);
    }
}

template <int B> static hipError_t launch_integrate_b(const IntegrateArgs &a, int n_groups,
                                                    int block_threads, hipStream_t s)
{
    size_t lds = (size_t)B * block_threads * sizeof(float);
    hipLaunchKernelGGL(integrate_kernel<B>, dim3(n_groups), dim3(block_threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_integrate(const IntegrateArgs &a, int n_groups, int block_threads, hipStream_t s)
{
    switch (a.block) {
    case 1: return launch_integrate_b<1>(a, n_groups, block_threads, s);
    case 2: return launch_integrate_b<2>(a, n_groups, block_threads, s);
    case 4: return launch_integrate_b<4>(a, n_groups, block_threads, s);
    case 8: return launch_integrate_b<8>(a, n_groups, block_threads, s);
    case 16: return launch_integrate_b<16>(a, n_groups, block_threads, s);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ FC and statistics
// One workgroup per instance. Rates are shifted by the first sample of each
// region (exact in FP64), then: per-region sums and sums of squares; the Gram
// matrix of the shifted samples over 4x4 tiles of the upper triangle, staged
// through LDS in chunks of samples; covariance, Pearson FC, and the statistics.
constexpr int kFcThreads = 256;
constexpr int kFcLdsFloats = 8192;

__device__ __forceinline__ double block_sum(double v, double *red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = kFcThreads / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kFcThreads) void fc_stats_kernel(FcArgs a)
{
    __shared__ float xs[kFcLdsFloats];
    __shared__ double shift[1024], mean[1024], var[1024];
    __shared__ double red[kFcThreads];
    const int64_t inst = blockIdx.x;
    const InstDev I = a.inst[inst];
    const ConnDev C = a.conns[I.conn];
    const int n = I.n, tid = threadIdx.x;
    const int64_t ns = a.n_samples;
    const float *x = a.ws + I.samp_off;
    const double *sc = a.sc + C.sc_off;
    float *fc = a.ws + I.fc_off;
    const double inv_ns = ns > 0 ? 1.0 / (double)ns : 0.0;

    // per-region moments
    for (int k = tid; k < n; k += kFcThreads) {
        double sh = ns > 0 ? (double)x[k] : 0.0, s1 = 0.0, s2 = 0.0;
        for (int64_t s = 0; s < ns; ++s) {
            double v = (double)x[s * n + k] - sh;
            s1 += v;
            s2 = fma(v, v, s2);
        }
        double m1 = s1 * inv_ns;
        shift[k] = sh;
        mean[k] = m1;   // mean of the shifted samples
        const double vk = ns > 0 ? s2 * inv_ns - m1 * m1 : 0.0;
        var[k] = vk < a.min_var ? 0.0 : vk;   // silent regions: zero variance
    }
    __syncthreads();

    const int nT = (n + 3) / 4, npad = nT * 4;
    const int ntiles = nT * (nT + 1) / 2;
    const int chunk = kFcLdsFloats / npad;
    double s_f = 0, s_f2 = 0, s_w = 0, s_w2 = 0, s_fw = 0, s_cov = 0;
    for (int t0 = 0; t0 < ntiles; t0 += kFcThreads) {
        const int t = t0 + tid;
        int tr = 0, tcol = 0;
        if (t < ntiles) {
            int rem = t;
            while (rem >= nT - tr) { rem -= nT - tr; ++tr; }
            tcol = tr + rem;
        }
        double P[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) P[i][j] = 0.0;
        for (int64_t s0 = 0; s0 < ns; s0 += chunk) {
            const int cn = (int)((ns - s0) < chunk ? (ns - s0) : chunk);
            __syncthreads();
            for (int i = tid; i < cn * npad; i += kFcThreads) {
                const int s = i / npad, k = i - s * npad;
                xs[i] = k < n ? x[(s0 + s) * n + k] : 0.f;
            }
            __syncthreads();
            if (t < ntiles) {
                double sa[4], sb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int ka = tr * 4 + i, kb = tcol * 4 + i;
                    sa[i] = ka < n ? shift[ka] : 0.0;
                    sb[i] = kb < n ? shift[kb] : 0.0;
                }
                for (int s = 0; s < cn; ++s) {
                    const float *row = xs + s * npad;
                    double va[4], vb[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        va[i] = (double)row[tr * 4 + i] - sa[i];
                        vb[i] = (double)row[tcol * 4 + i] - sb[i];
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) P[i][j] = fma(va[i], vb[j], P[i][j]);
                }
            }
        }
        if (t < ntiles) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = tr * 4 + i, l = tcol * 4 + j;
                    if (k >= n || l >= n || (tr == tcol && l < k)) continue;
                    if (k == l) {
                        fc[(int64_t)k * n + k] = 1.f;
                        s_cov += var[k];
                        continue;
                    }
                    const double cov = (var[k] > 0.0 && var[l] > 0.0)
                                           ? P[i][j] * inv_ns - mean[k] * mean[l] : 0.0;
                    const double f = (var[k] > 0.0 && var[l] > 0.0) ? cov / sqrt(var[k] * var[l])
                                                                    : 0.0;
                    fc[(int64_t)k * n + l] = (float)f;
                    fc[(int64_t)l * n + k] = (float)f;
                    const double wv = sc[(int64_t)k * n + l];
                    s_f += f;
                    s_f2 = fma(f, f, s_f2);
                    s_w += wv;
                    s_w2 = fma(wv, wv, s_w2);
                    s_fw = fma(f, wv, s_fw);
                    s_cov += 2.0 * cov;
                }
        }
    }
    double s_mean = 0, s_std = 0, s_var = 0;
    uint32_t zero_var = 0;
    for (int k = tid; k < n; k += kFcThreads) {
        s_mean += shift[k] + mean[k];
        s_std += sqrt(var[k] > 0.0 ? var[k] : 0.0);
        s_var += var[k];
        zero_var |= (var[k] > 0.0) ? 0u : 1u;
    }
    s_f = block_sum(s_f, red);
    s_f2 = block_sum(s_f2, red);
    s_w = block_sum(s_w, red);
    s_w2 = block_sum(s_w2, red);
    s_fw = block_sum(s_fw, red);
    s_cov = block_sum(s_cov, red);
    s_mean = block_sum(s_mean, red);
    s_std = block_sum(s_std, red);
    s_var = block_sum(s_var, red);
    const double zv = block_sum((double)zero_var, red);
    if (tid == 0) {
        const double cnt = 0.5 * (double)n * (double)(n - 1);
        const double mf = s_f / cnt;
        const double vf = s_f2 - s_f * s_f / cnt, vw = s_w2 - s_w * s_w / cnt;
        const double cfw = s_fw - s_f * s_w / cnt;
        float *st = a.stats + inst * 8;
        st[0] = (float)mf;
        st[1] = (float)sqrt(vf > 0.0 ? vf / cnt : 0.0);
        st[2] = (float)((vf > 0.0 && vw > 0.0) ? cfw / sqrt(vf * vw) : 0.0);
        st[3] = (float)(1000.0 * s_mean / n);
        st[4] = (float)(1000.0 * s_std / n);
        st[5] = (float)(s_var > 0.0 ? sqrt((s_cov / ((double)n * n)) / (s_var / n)) : 0.0);
        uint32_t flags = a.flags[inst] | (zv > 0.0 ? 4u : 0u);
        ((uint32_t *)st)[6] = flags;
        ((uint32_t *)st)[7] = 0u;
    }
}

hipError_t launch_fc_stats(const FcArgs &a, int64_t n_inst, hipStream_t s)
{
    if (n_inst == 0) return hipSuccess;
    hipLaunchKernelGGL(fc_stats_kernel, dim3((unsigned)n_inst), dim3(kFcThreads), 0, s, a);
    return hipGetLastError();
}

} // namespace vadx
