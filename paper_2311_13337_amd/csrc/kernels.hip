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
#include "philox.h"

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
// Philox4x32-10 is in philox.h.

// Four standard normals for steps 4q .. 4q+3 of region k: words mapped to
// (0, 1) as (w + 1/2) 2^-32, two Box-Muller (cos, sin) pairs. The hardware
// sine/cosine take their argument in revolutions, so sin(2 pi u) is one
// instruction; log2 and sqrt are the hardware instructions as well.
__device__ __forceinline__ void normals4(uint32_t seed, uint32_t id, uint32_t q, uint32_t k,
                                         float z[4])
{
    uint32_t c[4] = {q, k, 0u, 0u};
    philox4x32_10(c, seed, id);
    const float s32 = 2.3283064365386963e-10f, h32 = 1.1641532182693481e-10f;
    const float m2ln2 = -1.3862943611198906f;   // -2 ln 2
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const float u0 = fmaf((float)c[2 * p], s32, h32);
        const float u1 = fmaf((float)c[2 * p + 1], s32, h32);
        const float rr = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u0));
        z[2 * p] = rr * __builtin_amdgcn_cosf(u1);
        z[2 * p + 1] = rr * __builtin_amdgcn_sinf(u1);
    }
}

// ------------------------------------------------------------------ integrate
// Edges whose delayed histories a full block loads in one round of the
// coupling gather: about 96 floats in flight per lane for blocks of 24 and 32
// steps, 64 for shorter ones (measured: 6 edges of 16 steps ran slower than 4).
template <int B> constexpr int kGatherFloats = B > 16 ? 96 : 64;
template <int B> constexpr int kGatherEdges =
    B >= kGatherFloats<B> ? 1 : (kGatherFloats<B> / B > 8 ? 8 : kGatherFloats<B> / B);

// Waits until every wave in [lo, hi] other than `self` has published m
// steps of the current item (per-wave counters in LDS), then acquires their
// history writes. The wait is bounded: on timeout bit 1 of *status is set
// and the wave goes on (its results are then void, and the run reports it),
// so no wave can wait forever. Every argument is wave-uniform.
__device__ __forceinline__ void wait_waves(const int *wdone, int lo, int hi, int self, int m,
                                           uint32_t *status, uint32_t max_spins)
{
    for (int v = lo; v <= hi; ++v) {
        if (v == self) continue;
        uint32_t spins = 0;
        while (__builtin_amdgcn_readfirstlane(
                   __hip_atomic_load(&wdone[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) < m) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > max_spins) {
                if ((threadIdx.x & 63) == 0) atomicOr(status, 2u);
                break;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Integrates the instances of group g over steps [n_begin, n_end). All
// threads of the workgroup call it with the same (wave-uniform) arguments: it
// starts with a workgroup barrier. Inside, waves synchronise only with the
// waves that share an instance with them: each wave publishes the number of
// steps whose rates it has written (counters in LDS, `wdone`), and before the
// gather of the block from step s it waits until those waves have written
// slot s + B - 1 - d_min (the newest its reads reach, d_min the group's
// shortest delay). Waves thus drift up to d_min + 1 - B steps apart instead of
// meeting at a barrier after every block; the ring depth (d_max + d_min + 2)
// keeps a wave's writes clear of every slot a wave that far behind still
// reads.
//
template <int B, int VAR>
__device__ __forceinline__ void integrate_group(const IntegrateArgs &a, const GroupDev g,
                                                int64_t n_begin, int64_t n_end, float *cbuf,
                                                int *wdone)
{
    const int tid = threadIdx.x;
    const int slot = tid / g.n;
    const int k = tid - slot * g.n;
    const bool active = slot < g.count;
    const int nthr = blockDim.x;
    // this wave and the waves holding lanes of the instances it holds
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int used = g.count * g.n;
    const bool wave_live = wave * 64 < used;
    int wlo = wave, whi = wave - 1;
    if (wave_live) {
        const int last = (wave * 64 + 63 < used ? wave * 64 + 63 : used - 1) / g.n;
        wlo = ((wave * 64) / g.n * g.n) >> 6;
        whi = ((last + 1) * g.n - 1) >> 6;
    }
    if ((tid & 63) == 0) wdone[wave] = 0;

    InstDev I;
    double X[8];
    float acc = 0.f;
    int row_b = 0, row_e = 0;
    const float *wrow = nullptr;
    const int32_t *prow = nullptr;
    float *ring = nullptr;
    float *trace = nullptr;
    int tc = 0, sidx = 0;
    uint32_t fl = 0;
    const int tavg = (int)a.tavg_steps;
    const int ns = (int)a.n_samples;
    if (active) {
        I = a.inst[a.perm[g.first + slot]];
        const ConnDev C = a.conns[I.conn];
        row_b = a.rowptr[C.row_off + k];
        row_e = a.rowptr[C.row_off + k + 1];
        wrow = a.weight + C.edge_off;
        prow = a.packed + I.table_off;
        ring = a.ws + I.ring_off;
        if (I.trace_off >= 0) trace = a.ws + I.trace_off;
        tc = (int)(n_begin % tavg);
        sidx = (int)(n_begin / tavg - a.transient_steps / tavg);
        if (n_begin == 0) {
            X[0] = a.E_init;
            X[1] = a.I_init;
#pragma unroll
            for (int q = 2; q < 8; ++q) X[q] = 0.0;
            float *rr = ring + (int64_t)k * I.Dp;
            const float e0 = (float)a.E_init;
            for (int s = 0; s < I.Dp; ++s) rr[s] = e0;
        } else {
            const double *st = reinterpret_cast<const double *>(a.ws + I.state_off);
#pragma unroll
            for (int q = 0; q < 8; ++q) X[q] = st[q * I.n + k];
            acc = a.ws[I.acc_off + k];
        }
    }
    __syncthreads();   // initial rings and the wave counters visible to all lanes

    const float S = active ? I.S : 0.f;
    InstModel<float> P;
    P.be = active ? I.be : 0.f;
    P.ae = active ? I.ae : 0.f;
    P.w_noise = active ? I.w_noise : 0.f;
    P.inv_tauw_e = active ? I.inv_tauw_e : 0.f;
    P.cF[0][0] = active ? I.cF[0] : 0.f;
    P.cF[0][1] = active ? I.cF[1] : 0.f;
    P.cF[1][0] = active ? I.cF[2] : 0.f;
    P.cF[1][1] = active ? I.cF[3] : 0.f;
    const KModel M = *a.Mp;
    const int D = active ? I.D : 1;
    const int Dp = active ? I.Dp : 1;
    int nm = active ? (int)(n_begin % D) : 0;   // n0 mod D
    float *myrow = active ? ring + (int64_t)k * Dp : nullptr;
    float z4[4] = {0.f, 0.f, 0.f, 0.f};

    for (int64_t n0 = n_begin; n0 < n_end && wave_live; n0 += B) {
        const int nb = (int)((n_end - n0) < B ? (n_end - n0) : B);
        // steps of this item the other waves must have published: the block
        // reads slots up to n0 + B - 1 - d_min (earlier items' slots are all written)
        const int need = (int)(n0 - n_begin) + B - 1 - g.dmin;
        if (need > 0) wait_waves(wdone, wlo, whi, wave, need, a.status, a.wait_spins);
        if (active) {
            // coupling of steps n0 .. n0+nb-1: S sum_j W_kj H_j[n - d_kj], in the
            // fixed (ascending j) order of the CSR row
            float cb[B];
#pragma unroll
            for (int b = 0; b < B; ++b) cb[b] = 0.f;
            if (nb == B) {
                // kGatherEdges edges per round, without branches: the round's
                // history loads are all in flight before its first multiply-add,
                // and the next round's edge indices and weights are loaded while
                // they are, so a round costs one memory round trip. Past the
                // row's end a round re-reads the row's last edge with weight 0.
                // The sums run over the edges in row order. Offsets stay in 32
                // bits: j < 512 regions and ring rows under 2^21 + 32 slots, so
                // j * Dp fits the 24-bit multiplier and the offset an int.
                constexpr int U = kGatherEdges<B>;
                // the row bounds pass through an empty asm so that the first
                // round's addresses are formed here, each block, instead of
                // being hoisted out of the block loop and kept (spilled) across
                // the steps
                int rb = row_b, re = row_e;
                asm volatile("" : "+v"(rb), "+v"(re));
                const int last = re - 1;
                int32_t pk[U];
                float w[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    // an empty row loads nothing (its first index may be the
                    // table's end)
                    const int e = min(rb + u, last);
                    pk[u] = rb < re ? prow[e] : 0;
                    w[u] = rb < re ? wrow[e] : 0.f;
                }
                for (int e0 = rb; e0 < re; e0 += U) {
                    const float *h[U];
                    float wc[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int j = pk[u] >> 20, d = pk[u] & 0xFFFFF;
                        int s0 = nm - d;
                        s0 += (s0 < 0) ? D : 0;
                        h[u] = ring + (__umul24((uint32_t)j, (uint32_t)Dp) + (uint32_t)s0);
                        wc[u] = e0 + u < re ? w[u] : 0.f;
                    }
                    float hv[U][B];
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int b = 0; b < B; ++b) hv[u][b] = h[u][b];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int e = min(e0 + U + u, last);
                        pk[u] = prow[e];
                        w[u] = wrow[e];
                    }
                    // keep those loads here, ahead of the waits for the histories
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int b = 0; b < B; ++b) cb[b] = fmaf(wc[u], hv[u][b], cb[b]);
                }
            } else {
                for (int e = row_b; e < row_e; ++e) {
                    const int32_t pk = prow[e];
                    const int j = pk >> 20, d = pk & 0xFFFFF;
                    const float w = wrow[e];
                    int s0 = nm - d;
                    s0 += (s0 < 0) ? D : 0;
                    const float *h = ring + (int64_t)j * Dp + s0;
#pragma unroll
                    for (int b = 0; b < B; ++b)
                        if (b < nb) cb[b] = fmaf(w, h[b], cb[b]);
                }
            }
#pragma unroll
            for (int b = 0; b < B; ++b) cbuf[b * nthr + tid] = S * cb[b];

            const bool tracing = trace != nullptr && n0 < a.n_trace_steps;
            for (int b = 0; b < nb; ++b) {
                const int n = (int)(n0 + b);
                const int r = n & 3;
                if (r == 0 || b == 0)
                    normals4(a.seed, I.id, (uint32_t)(n >> 2), (uint32_t)k, z4);
                const float z = r == 0 ? z4[0] : (r == 1 ? z4[1] : (r == 2 ? z4[2] : z4[3]));
                const float c = cbuf[b * nthr + tid];
                fl |= step_region<VAR>(M, a.integrator, a.dt, X, c, P,
                                       a.gdw_scale * (double)z);
                // the new E waits in this step's coupling slot, which is free
                // now, and goes to the history ring at the end of the block
                const float e1 = (float)X[0];
                cbuf[b * nthr + tid] = e1;
                // time average
                acc += e1;
                if (++tc == tavg) {
                    if (sidx >= 0 && sidx < ns)
                        a.ws[I.samp_off + (int64_t)sidx * I.n + k] = acc / (float)tavg;
                    acc = 0.f;
                    tc = 0;
                    ++sidx;
                }
                if (tracing && n < a.n_trace_steps) {
                    float *tr = trace + (int64_t)n * 8 * I.n + k;
#pragma unroll
                    for (int q = 0; q < 8; ++q) tr[q * I.n] = (float)X[q];
                }
            }
            // history of E for steps n0+1 .. n0+nb: slots (n0 + 1 + b) mod D, and
            // the mirrors D + t of slots t < B - 1, written as one run per lane
            // (nothing reads them before the block is published)
            int t0 = nm + 1;
            t0 -= (t0 >= D) ? D : 0;
            if (nb == B && t0 + B <= D) {
                float eb[B];
#pragma unroll
                for (int b = 0; b < B; ++b) eb[b] = cbuf[b * nthr + tid];
#pragma unroll
                for (int b = 0; b < B; ++b) myrow[t0 + b] = eb[b];
                if (t0 < B - 1) {
#pragma unroll
                    for (int b = 0; b < B - 1; ++b)
                        if (t0 + b < B - 1) myrow[D + t0 + b] = eb[b];
                }
            } else {
                int t = t0;
                for (int b = 0; b < nb; ++b) {
                    const float e = cbuf[b * nthr + tid];
                    myrow[t] = e;
                    if (t < B - 1) myrow[D + t] = e;
                    t += 1;
                    t -= (t >= D) ? D : 0;
                }
            }
            nm += nb;
            nm -= (nm >= D) ? D : 0;
        }
        // publish this block's history to the waves that share its instances
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if ((tid & 63) == 0)
            __hip_atomic_store(&wdone[wave], (int)(n0 + nb - n_begin), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (active) {
        double *st = reinterpret_cast<double *>(a.ws + I.state_off);
#pragma unroll
        for (int q = 0; q < 8; ++q) st[q * I.n + k] = X[q];
        a.ws[I.acc_off + k] = acc;
        if (fl) atomicOr(&a.flags[a.perm[g.first + slot]], fl);
    }
}

template <int B, int VAR>
__global__ __launch_bounds__(512) void integrate_kernel(IntegrateArgs a)
{
    extern __shared__ float cbuf[];   // [B][blockDim.x] coupling of the block's steps
    __shared__ int wdone[8];
    integrate_group<B, VAR>(a, a.groups[blockIdx.x], a.n_begin, a.n_end, cbuf, wdone);
}

// One group over [n_begin, n_end) with the group's own block length.
template <int VAR>
__device__ __forceinline__ void integrate_group_any(const IntegrateArgs &a, const GroupDev g,
                                                    int64_t n_begin, int64_t n_end, float *cbuf,
                                                    int *wdone)
{
    switch (g.block) {
    case 1: integrate_group<1, VAR>(a, g, n_begin, n_end, cbuf, wdone); break;
    case 2: integrate_group<2, VAR>(a, g, n_begin, n_end, cbuf, wdone); break;
    case 4: integrate_group<4, VAR>(a, g, n_begin, n_end, cbuf, wdone); break;
    case 8: integrate_group<8, VAR>(a, g, n_begin, n_end, cbuf, wdone); break;
    case 12: integrate_group<12, VAR>(a, g, n_begin, n_end, cbuf, wdone); break;
    case 16: integrate_group<16, VAR>(a, g, n_begin, n_end, cbuf, wdone); break;
    case 24: integrate_group<24, VAR>(a, g, n_begin, n_end, cbuf, wdone); break;
    default: integrate_group<32, VAR>(a, g, n_begin, n_end, cbuf, wdone); break;
    }
}

// Persistent form: workgroups pull (group, chunk) items from a queue in
// chunk-major order over the groups of every block length, so one launch
// integrates a whole uneven batch; each group runs with its own block length
// and instance count. Chunk c of a group starts only after chunk c-1 of the
// same group has been published (its state and history written back to
// memory), so the groups advance in step while every workgroup stays busy
// until the queue is empty. The wait is bounded: on timeout the kernel
// records an error and the workgroup stops.
// OCC: waves per SIMD the register allocation must allow (2: one 512-lane or
// two 256-lane workgroups per CU, no spills; 3: three 256-lane workgroups, a
// few spills outside the step loop). (A budget of 4 waves, 128 registers,
// spills inside the step loop and measured slower than both.)
template <int VAR, int OCC>
__global__ __launch_bounds__(512, OCC) void integrate_persistent_kernel(IntegrateArgs a, QueueArgs q)
{
    extern __shared__ float cbuf[];   // [largest block][blockDim.x]
    __shared__ int wdone[8];
    __shared__ int s_item;
    __shared__ int s_abort;
    const int tid = threadIdx.x;
    const int G = q.n_groups;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(q.next, 1);
        __syncthreads();
        // Every value that steers loops and barriers below is made wave-uniform
        // (scalar): with an LDS-loaded index the compiler treats the loop exits
        // as divergent and may restructure the loop so that waves reach the
        // workgroup barriers in different orders.
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();                           // s_item read by all before it is rewritten
        if (item >= q.n_items) break;
        const int c = item / G, gi = item - c * G;
        if (c > 0) {
            if (tid == 0) {
                uint32_t spins = 0;
                int abort = 0;
                while (__hip_atomic_load(&q.done[gi], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < c) {
                    __builtin_amdgcn_s_sleep(32);
                    if (++spins > q.max_spins) {
                        atomicOr(q.status, 1u);
                        abort = 1;
                        break;
                    }
                }
                s_abort = abort;
            }
            __syncthreads();
            const int abort = __builtin_amdgcn_readfirstlane(s_abort);
            if (abort) break;
            __atomic_thread_fence(__ATOMIC_ACQUIRE);   // see the previous chunk's writes
        }
        const int64_t nb = a.n_begin + (int64_t)c * q.item_steps;
        const int64_t ne = nb + q.item_steps < a.n_end ? nb + q.item_steps : a.n_end;
        integrate_group_any<VAR>(a, a.groups[gi], nb, ne, cbuf, wdone);
        __threadfence();                           // publish state and history
        __syncthreads();
        if (tid == 0)
            __hip_atomic_store(&q.done[gi], c + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Clears n words (a kernel rather than a memset node, so a captured run
// graph holds kernels only).
__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t value, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

// Stores the run's model constants where the integration kernels read them
// (once per queue item, from device memory, rather than holding them in
// scalar registers for the whole launch).
__global__ void kmodel_store_kernel(KModel m, KModel *out)
{
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&m);
    uint32_t *dst = reinterpret_cast<uint32_t *>(out);
    for (int i = threadIdx.x; i < (int)(sizeof(KModel) / 4); i += blockDim.x) dst[i] = src[i];
}

hipError_t launch_kmodel_store(const KModel &m, KModel *out, hipStream_t s)
{
    hipLaunchKernelGGL(kmodel_store_kernel, dim3(1), dim3(64), 0, s, m, out);
    return hipGetLastError();
}

__global__ void queue_reset_kernel(QueueArgs q)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *q.next = 0;
    if (i < q.n_groups) q.done[i] = 0;
}

template <int B, int VAR>
static hipError_t launch_integrate_b(const IntegrateArgs &a, int n_groups, int block_threads,
                                     hipStream_t s)
{
    size_t lds = (size_t)B * block_threads * sizeof(float);
    hipLaunchKernelGGL((integrate_kernel<B, VAR>), dim3(n_groups), dim3(block_threads), lds, s, a);
    return hipGetLastError();
}

template <int VAR>
static hipError_t launch_integrate_v(const IntegrateArgs &a, int n_groups, int block_threads,
                                     hipStream_t s)
{
    switch (a.block) {
    case 1: return launch_integrate_b<1, VAR>(a, n_groups, block_threads, s);
    case 2: return launch_integrate_b<2, VAR>(a, n_groups, block_threads, s);
    case 4: return launch_integrate_b<4, VAR>(a, n_groups, block_threads, s);
    case 8: return launch_integrate_b<8, VAR>(a, n_groups, block_threads, s);
    case 12: return launch_integrate_b<12, VAR>(a, n_groups, block_threads, s);
    case 16: return launch_integrate_b<16, VAR>(a, n_groups, block_threads, s);
    case 24: return launch_integrate_b<24, VAR>(a, n_groups, block_threads, s);
    case 32: return launch_integrate_b<32, VAR>(a, n_groups, block_threads, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_integrate(const IntegrateArgs &a, int n_groups, int block_threads, hipStream_t s)
{
    switch (model_variant(a.M)) {
    case 0: return launch_integrate_v<0>(a, n_groups, block_threads, s);
    case 1: return launch_integrate_v<1>(a, n_groups, block_threads, s);
    case 2: return launch_integrate_v<2>(a, n_groups, block_threads, s);
    default: return launch_integrate_v<3>(a, n_groups, block_threads, s);
    }
}

template <int VAR, int OCC>
static hipError_t launch_persistent_v(const IntegrateArgs &a, int block_threads, const QueueArgs &q,
                                      int grid, hipStream_t s)
{
    hipLaunchKernelGGL(queue_reset_kernel, dim3((q.n_groups + 255) / 256), dim3(256), 0, s, q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t lds = (size_t)a.block * block_threads * sizeof(float);
    hipLaunchKernelGGL((integrate_persistent_kernel<VAR, OCC>), dim3(grid), dim3(block_threads),
                       lds, s, a, q);
    return hipGetLastError();
}

template <int OCC>
static hipError_t launch_persistent_o(const IntegrateArgs &a, int block_threads, const QueueArgs &q,
                                      int grid, hipStream_t s)
{
    switch (model_variant(a.M)) {
    case 0: return launch_persistent_v<0, OCC>(a, block_threads, q, grid, s);
    case 1: return launch_persistent_v<1, OCC>(a, block_threads, q, grid, s);
    case 2: return launch_persistent_v<2, OCC>(a, block_threads, q, grid, s);
    default: return launch_persistent_v<3, OCC>(a, block_threads, q, grid, s);
    }
}

hipError_t launch_integrate_persistent(const IntegrateArgs &a, int block_threads, const QueueArgs &q,
                                       int grid, int occ, hipStream_t s)
{
    if (occ == 3) return launch_persistent_o<3>(a, block_threads, q, grid, s);
    return launch_persistent_o<2>(a, block_threads, q, grid, s);
}

template <int OCC> static int resident_o(int max_block, int block_threads)
{
    // all model variants have the same launch bounds and LDS use
    int per_cu = 1 << 30;
    size_t lds = (size_t)max_block * block_threads * sizeof(float);
    void (*kernels[4])(IntegrateArgs, QueueArgs) = {
        integrate_persistent_kernel<0, OCC>, integrate_persistent_kernel<1, OCC>,
        integrate_persistent_kernel<2, OCC>, integrate_persistent_kernel<3, OCC>};
    for (auto k : kernels) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, block_threads, lds) != hipSuccess)
            return 0;
        per_cu = n < per_cu ? n : per_cu;
    }
    return per_cu;
}

int persistent_blocks_per_cu(int max_block, int block_threads, int occ)
{
    if (occ == 3) return resident_o<3>(max_block, block_threads);
    return resident_o<2>(max_block, block_threads);
}

// ------------------------------------------------------------------ FC and statistics
// One workgroup per instance. Rates are shifted by the first sample of each
// region (exact in FP64) and staged through LDS in FP64, in chunks of
// samples; from them, per-region sums and sums of squares and the Gram matrix
// over 4x4 tiles of the upper triangle; then covariance, Pearson FC, and the
// statistics.
constexpr int kFcThreads = 256;
constexpr int kFcStageDoubles = 4096;    // shifted samples staged per chunk (32 KB)
constexpr int kFcRegionsPerThread = 4;   // regions per thread in the moment sums (n <= 1024)
constexpr int kFcStagePerThread = kFcStageDoubles / kFcThreads;   // staged samples per thread

// Dynamic LDS of fc_stats_kernel for instances of up to max_n regions: the
// staged samples, shift / mean / variance per region, a reduction buffer.
size_t fc_lds_bytes(int max_n)
{
    return sizeof(double) * ((size_t)kFcStageDoubles + 3 * (size_t)max_n + kFcThreads);
}

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

__global__ __launch_bounds__(kFcThreads, 4) void fc_stats_kernel(FcArgs a)
{
    extern __shared__ __align__(16) double fcl[];   // fc_lds_bytes(a.max_n)
    double *xs = fcl;                                // [chunk][npad] shifted samples
    double *shift = xs + kFcStageDoubles, *mean = shift + a.max_n, *var = mean + a.max_n;
    double *red = var + a.max_n;
    const int64_t inst = blockIdx.x;
    const InstDev I = a.inst[inst];
    const ConnDev C = a.conns[I.conn];
    const int n = I.n, tid = threadIdx.x;
    const int64_t ns = a.n_samples;
    const float *x = a.ws + I.samp_off;
    const double *sc = a.sc + C.sc_off;
    const float *ref = C.ref_off >= 0 ? a.ref + C.ref_off : nullptr;
    float *fc = a.ws + I.fc_off;
    const double inv_ns = ns > 0 ? 1.0 / (double)ns : 0.0;

    // shifts: the first sample of each region (exact in FP64)
    for (int k = tid; k < n; k += kFcThreads) shift[k] = ns > 0 ? (double)x[k] : 0.0;
    __syncthreads();

    const int nT = (n + 3) / 4, npad = nT * 4;
    const int ntiles = nT * (nT + 1) / 2;
    const int chunk = kFcStageDoubles / npad;
    // e / npad for e < kFcStageDoubles as (e + 1/2) times the rounded
    // reciprocal, truncated: the quotient stays at least 1/(2 npad) from an
    // integer, its rounding error below e 2^-23 / npad, so the row is exact
    const float inv_npad = 1.f / (float)npad;
    double s_f = 0, s_f2 = 0, s_w = 0, s_w2 = 0, s_fw = 0, s_cov = 0;
    double s_r = 0, s_r2 = 0, s_fr = 0;           // reference FC (fitness)
    // per-region sums of the shifted samples and of their squares, gathered
    // from the LDS-staged samples during the first pass over the tiles
    double m1[kFcRegionsPerThread], m2[kFcRegionsPerThread];
#pragma unroll
    for (int q = 0; q < kFcRegionsPerThread; ++q) m1[q] = m2[q] = 0.0;
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
            // stage the chunk: element e = s npad + k (sample s, region k) of
            // the LDS block comes from x[(s0 + s) n + k]; a thread issues all
            // its loads before storing any
            const int ne = cn * npad;
            const float *xc = x + s0 * n;
            float v[kFcStagePerThread];
#pragma unroll
            for (int j = 0; j < kFcStagePerThread; ++j) {
                const int e = tid + j * kFcThreads;
                const int sj = (int)(((float)e + 0.5f) * inv_npad), kj = e - sj * npad;
                // unconditional loads (elements outside the chunk or in the
                // padding read the chunk's first sample, unused)
                v[j] = xc[(e < ne && kj < n) ? sj * n + kj : 0];
            }
            __syncthreads();
            // the stores re-derive the indices from an opaque copy of tid, so
            // that only the loaded values stay live between the two loops
            int tid2 = tid;
            asm volatile("" : "+v"(tid2));
#pragma unroll
            for (int j = 0; j < kFcStagePerThread; ++j) {
                const int e = tid2 + j * kFcThreads;
                const int sj = (int)(((float)e + 0.5f) * inv_npad), kj = e - sj * npad;
                if (e < ne) xs[e] = kj < n ? (double)v[j] - shift[kj] : 0.0;
            }
            __syncthreads();
            if (t0 == 0) {
#pragma unroll
                for (int q = 0; q < kFcRegionsPerThread; ++q) {
                    const int k = tid + q * kFcThreads;
                    if (k < n) {
                        for (int s = 0; s < cn; ++s) {
                            const double v = xs[s * npad + k];
                            m1[q] += v;
                            m2[q] = fma(v, v, m2[q]);
                        }
                    }
                }
            }
            if (t < ntiles) {
                for (int s = 0; s < cn; ++s) {
                    const double *row = xs + s * npad;
                    double va[4], vb[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        va[i] = row[tr * 4 + i];
                        vb[i] = row[tcol * 4 + i];
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) P[i][j] = fma(va[i], vb[j], P[i][j]);
                }
            }
        }
        if (t0 == 0) {
            // moments complete: means of the shifted samples and variances
#pragma unroll
            for (int q = 0; q < kFcRegionsPerThread; ++q) {
                const int k = tid + q * kFcThreads;
                if (k < n) {
                    const double mk = m1[q] * inv_ns;
                    mean[k] = mk;
                    const double vk = ns > 0 ? m2[q] * inv_ns - mk * mk : 0.0;
                    var[k] = vk < a.min_var ? 0.0 : vk;   // silent regions: zero variance
                }
            }
            __syncthreads();
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
                    if (ref) {
                        const double rv = (double)ref[(int64_t)k * n + l];
                        s_r += rv;
                        s_r2 = fma(rv, rv, s_r2);
                        s_fr = fma(f, rv, s_fr);
                    }
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
    if (ref) {
        s_r = block_sum(s_r, red);
        s_r2 = block_sum(s_r2, red);
        s_fr = block_sum(s_fr, red);
    }
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
        // fitness: Pearson correlation of FC_kl with the reference over k < l
        const double vr = s_r2 - s_r * s_r / cnt, cfr = s_fr - s_f * s_r / cnt;
        st[7] = (float)((ref && vf > 0.0 && vr > 0.0) ? cfr / sqrt(vf * vr) : 0.0);
    }
}

// Orders k (value, index) pairs by decreasing value, ties by increasing index:
// each pair's output position is the number of pairs that precede it.
constexpr int kRankMax = 1024;
__global__ __launch_bounds__(kRankMax) void rank_sort_kernel(const float *val, const int64_t *idx,
                                                             int32_t k, int64_t *idx_out,
                                                             float *val_out)
{
    __shared__ float v[kRankMax];
    __shared__ int64_t ix[kRankMax];
    const int t = threadIdx.x;
    if (t < k) {
        v[t] = val[idx[t]];
        ix[t] = idx[t];
    }
    __syncthreads();
    if (t < k) {
        int r = 0;
        for (int j = 0; j < k; ++j)
            r += (v[j] > v[t] || (v[j] == v[t] && ix[j] < ix[t])) ? 1 : 0;
        idx_out[r] = ix[t];
        if (val_out) val_out[r] = v[t];
    }
}

hipError_t launch_rank_sort(const float *val, const int64_t *idx, int32_t k, int64_t *idx_out,
                            float *val_out, hipStream_t s)
{
    if (k <= 0) return hipSuccess;
    if (k > kRankMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(rank_sort_kernel, dim3(1), dim3(kRankMax), 0, s, val, idx, k, idx_out,
                       val_out);
    return hipGetLastError();
}

hipError_t launch_fc_stats(const FcArgs &a, int64_t n_inst, hipStream_t s)
{
    if (n_inst == 0) return hipSuccess;
    if (a.max_n < 1 || a.max_n > 1024) return hipErrorInvalidValue;
    const size_t lds = fc_lds_bytes(a.max_n);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fc_stats_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fc_stats_kernel, dim3((unsigned)n_inst), dim3(kFcThreads), lds, s, a);
    return hipGetLastError();
}


} // namespace vadx
