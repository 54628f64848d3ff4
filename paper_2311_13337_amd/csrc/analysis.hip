// analysis.hip -- the analysis metrics of Section 2.6 (Table 2) over stored
// excitatory rate samples: a transpose of each instance's analysis window to
// time-contiguous rows, Welch power spectra and analytic signals by FFTs in
// LDS, the phase lag index over region pairs, Up/Down state durations, and a
// per-instance reduction (spectrum peak, power-law fit, means).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "analysis_engine.h"

namespace vadx {

namespace {

__device__ inline float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cmulconj(float2 a, float2 b)   // a * conj(b)
{
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// Twiddle factors exp(-2 pi i j / kTwMax) from two LDS tables of kTwSplit
// entries: w(j) = hi[j / kTwSplit] * lo[j mod kTwSplit] (one rounding more
// than a full table, whose 128 KB would not fit beside the data).
constexpr int kTwSplit = 128;
static_assert(kTwSplit * kTwSplit == kTwMax, "two-level twiddle table");

struct TwLds {
    float2 lo[kTwSplit], hi[kTwSplit];
};

__device__ inline void load_twiddles(TwLds &t, const float2 *__restrict__ tw)
{
    for (int j = threadIdx.x; j < kTwSplit; j += blockDim.x) {
        t.lo[j] = tw[j];
        t.hi[j] = tw[j * kTwSplit];
    }
}

__device__ inline float2 twiddle(const TwLds &t, int j)
{
    return cmul(t.hi[j >> 7], t.lo[j & (kTwSplit - 1)]);
}

// Stockham autosort FFT over `batch` transforms of length N = 2^log2N stored
// back to back in LDS (batch * N <= NT * Q4 * 4): radix-4 stages, then one
// radix-2 stage when log2N is odd. Stage with sub-length Ns and radix R:
// butterfly j reads x[j + r N/R] (r < R), multiplies input r by
// w^(r (j mod Ns)) with w = exp(-+2 pi i / (Ns R)), applies the R-point DFT and
// writes output r to ((j div Ns) Ns R + j mod Ns + r Ns). Every thread holds its
// inputs in registers across a barrier, so input and output share the buffer.
// INV: the inverse transform (conjugate twiddles, no 1/N scaling).
template <int NT, int Q4, bool INV>
__device__ void fft_lds(float2 *buf, int log2N, int batch, const TwLds &tw)
{
    const int tid = threadIdx.x;
    const int N = 1 << log2N;
    const int total = N * batch;
    int Ns = 1, log2Ns = 0;
    for (; Ns * 4 <= N; Ns *= 4, log2Ns += 2) {
        const int quarter = N >> 2;
        const int nb = total >> 2;
        const int step = kTwMax >> (log2Ns + 2);
        float2 v[Q4][4];
#pragma unroll
        for (int q = 0; q < Q4; ++q) {
            const int j = tid + q * NT;
            if (j < nb) {
                const int b = j >> (log2N - 2), jj = j & (quarter - 1);
                const float2 *src = buf + (b << log2N) + jj;
                v[q][0] = src[0];
                v[q][1] = src[quarter];
                v[q][2] = src[2 * quarter];
                v[q][3] = src[3 * quarter];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q4; ++q) {
            const int j = tid + q * NT;
            if (j < nb) {
                const int b = j >> (log2N - 2), jj = j & (quarter - 1);
                const int k = jj & (Ns - 1);
                const float2 w1 = twiddle(tw, k * step);
                const float2 w2 = cmul(w1, w1), w3 = cmul(w2, w1);
                const float2 a0 = v[q][0];
                const float2 a1 = INV ? cmulconj(v[q][1], w1) : cmul(v[q][1], w1);
                const float2 a2 = INV ? cmulconj(v[q][2], w2) : cmul(v[q][2], w2);
                const float2 a3 = INV ? cmulconj(v[q][3], w3) : cmul(v[q][3], w3);
                const float2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
                const float2 s13 = cadd(a1, a3), d13 = csub(a1, a3);
                // forward: X1 = d02 - i d13, X3 = d02 + i d13 (inverse: signs swapped)
                const float2 r13 = INV ? make_float2(-d13.y, d13.x) : make_float2(d13.y, -d13.x);
                float2 *dst = buf + (b << log2N) + ((jj - k) << 2) + k;
                dst[0] = cadd(s02, s13);
                dst[Ns] = cadd(d02, r13);
                dst[2 * Ns] = csub(s02, s13);
                dst[3 * Ns] = csub(d02, r13);
            }
        }
        __syncthreads();
    }
    if (Ns < N) {                       // one radix-2 stage: Ns = N / 2
        const int half = N >> 1;
        const int nb = total >> 1;
        const int step = kTwMax >> (log2Ns + 1);
        float2 v[2 * Q4][2];
#pragma unroll
        for (int q = 0; q < 2 * Q4; ++q) {
            const int j = tid + q * NT;
            if (j < nb) {
                const int b = j >> (log2N - 1), jj = j & (half - 1);
                const float2 *src = buf + (b << log2N) + jj;
                v[q][0] = src[0];
                v[q][1] = src[half];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2 * Q4; ++q) {
            const int j = tid + q * NT;
            if (j < nb) {
                const int b = j >> (log2N - 1), k = j & (half - 1);
                const float2 w = twiddle(tw, k * step);
                const float2 a1 = INV ? cmulconj(v[q][1], w) : cmul(v[q][1], w);
                float2 *dst = buf + (b << log2N) + k;
                dst[0] = cadd(v[q][0], a1);
                dst[half] = csub(v[q][0], a1);
            }
        }
        __syncthreads();
    }
}

// Wave-wide sum in a fixed order (xor butterfly over the 64 lanes).
__device__ inline float wave_sum(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ inline float wave_min(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fminf(v, __shfl_xor(v, m, 64));
    return v;
}

__device__ inline float wave_max(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
    return v;
}

} // namespace

// ------------------------------------------------------------------ transpose
// Window of instance i ([Na][n] at the tail of its [n_samples][n] block) to
// rows xT[rbase + k][t]. A workgroup (256 threads) moves 64 samples of up to
// kTrRegions regions: with n <= kTrRegions that is one contiguous run of the
// source, read in order (consecutive threads, consecutive floats); each wave
// then writes 64-sample pieces (256 B) of its rows.
constexpr int kTrRegions = 128;
constexpr int kTrPerThread = 64 * kTrRegions / 256;   // tile elements per thread, at most

__global__ __launch_bounds__(256) void an_transpose_kernel(AnChunk a, int kchunks_max)
{
    __shared__ float tile[64][kTrRegions + 1];    // odd row pitch: column reads hit distinct banks
    const int i = blockIdx.y;
    const int n = a.n[i];
    const int kc = blockIdx.x % kchunks_max, tt = blockIdx.x / kchunks_max;
    const int k0 = kc * kTrRegions;
    if (k0 >= n) return;
    const int kw = min(kTrRegions, n - k0);
    const int t0 = tt * 64;
    const int rows = min(64, a.Na - t0);
    const float *src = a.samples + a.samp_off[i] + (a.n_samples - a.Na + t0) * (int64_t)n + k0;
    // thread tid takes tile elements e = tid + 256 j, row r = floor(e / kw),
    // column e - r kw: source offset e + r (n - kw), LDS offset e + r (pitch -
    // kw). All its loads are issued before the first is stored to LDS. r is
    // taken as (e + 1/2) times the rounded reciprocal of kw, truncated: for
    // e < 2^13 and kw <= 128 the quotient stays at least 1/256 from an integer
    // and its rounding error is below 1e-5, so r is exact.
    const float inv_kw = 1.f / (float)kw;
    const int ne = rows * kw;
    const uint32_t src_gap = (uint32_t)(n - kw), lds_gap = (uint32_t)(kTrRegions + 1 - kw);
    const float eh = (float)threadIdx.x + 0.5f;
    float v[kTrPerThread];
    uint32_t lo[kTrPerThread];
#pragma unroll
    for (int j = 0; j < kTrPerThread; ++j) {
        const uint32_t e = threadIdx.x + 256u * j;
        const uint32_t r = (uint32_t)((eh + (float)(256 * j)) * inv_kw);
        lo[j] = __umul24(r, lds_gap) + e;
        v[j] = (int)e < ne ? src[__umul24(r, src_gap) + e] : 0.f;
    }
    float *tflat = &tile[0][0];
#pragma unroll
    for (int j = 0; j < kTrPerThread; ++j)
        if ((int)(threadIdx.x + 256u * j) < ne) tflat[lo[j]] = v[j];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < rows) {
        float *dst = a.xT + (int64_t)(a.rbase[i] + k0) * a.Na + t0 + lane;
#pragma unroll 4
        for (int k = wave; k < kw; k += 4) dst[(int64_t)k * a.Na] = tile[lane][k];
    }
}

hipError_t launch_an_transpose(const AnChunk &a, int max_n, hipStream_t s)
{
    const int kchunks = (max_n + kTrRegions - 1) / kTrRegions;
    const int ttiles = (a.Na + 63) / 64;
    dim3 grid((unsigned)(kchunks * ttiles), (unsigned)a.n_inst);
    hipLaunchKernelGGL(an_transpose_kernel, grid, dim3(256), 0, s, a, kchunks);
    return hipGetLastError();
}

// ---------------------------------------------------------------------- Welch
// One workgroup per region. Each segment's mean is taken of its deviations
// from its first sample (a constant segment detrends to exact zeros). Segments
// 2p and 2p+1, detrended and windowed, form the real and imaginary parts of one
// complex transform Z; for real segments a, b the summed periodogram is
// |A_f|^2 + |B_f|^2 = (|Z_f|^2 + |Z_{L-f}|^2) / 2 (an odd last segment rides
// alone, with the same identity). Batches of such transforms run in LDS; each
// bin is owned by one thread, so the sum runs over segments in order.
constexpr int kWelchBinsPerThread = (kMaxSegment / 2 + 1 + kWelchThreads - 1) / kWelchThreads;
constexpr int kMaxSegments = 2 * kTwMax / kMinSegment;

__global__ __launch_bounds__(kWelchThreads) void an_welch_kernel(AnChunk a)
{
    extern __shared__ float2 buf[];               // kWelchBatch complex values
    __shared__ float smean[kMaxSegments];         // mean deviation from the segment's first sample
    __shared__ float smm[2][kWelchThreads / 64];  // per-wave min and max of the window
    __shared__ TwLds tw;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t g = blockIdx.x;
    const float *x = a.xT + g * a.Na;
    const int L = a.L, hop = L >> 1;
    const float invL = 1.f / (float)L;            // a power of two: exact
    load_twiddles(tw, a.tw);
    // the segments (hop L/2, (Na - L)/hop + 1 of them) cover the window
    // exactly, so the same pass takes the window's min and max for the
    // Up/Down kernel
    float wmn = INFINITY, wmx = -INFINITY;
    for (int sg = wave; sg < a.n_seg; sg += kWelchThreads / 64) {
        const float *xs = x + sg * hop;
        const float ref = xs[0];
        float s = 0.f;
#pragma unroll 4
        for (int m = lane; m < L; m += 64) {
            const float v = xs[m];
            s += v - ref;
            wmn = fminf(wmn, v);
            wmx = fmaxf(wmx, v);
        }
        s = wave_sum(s);
        if (lane == 0) smean[sg] = s * invL;
    }
    wmn = wave_min(wmn);
    wmx = wave_max(wmx);
    if (lane == 0) {
        smm[0][wave] = wmn;
        smm[1][wave] = wmx;
    }
    __syncthreads();
    if (tid == 0) {
        float mn = smm[0][0], mx = smm[1][0];
        for (int w = 1; w < kWelchThreads / 64; ++w) {
            mn = fminf(mn, smm[0][w]);
            mx = fmaxf(mx, smm[1][w]);
        }
        a.ud[g * 4] = __float_as_int(mn);
        a.ud[g * 4 + 1] = __float_as_int(mx);
    }
    const int nb2 = L / 2 + 1;
    float acc[kWelchBinsPerThread];
#pragma unroll
    for (int q = 0; q < kWelchBinsPerThread; ++q) acc[q] = 0.f;
    const int per_batch = kWelchBatch >> a.log2L;          // transforms per batch
    const int n_pairs = (a.n_seg + 1) >> 1;
    for (int p0 = 0; p0 < n_pairs; p0 += per_batch) {
        const int np = min(per_batch, n_pairs - p0);
#pragma unroll 4
        for (int e = tid; e < (np << a.log2L); e += kWelchThreads) {
            const int p = p0 + (e >> a.log2L), m = e & (L - 1);
            const int sa = 2 * p, sb = sa + 1;
            // an odd last segment rides alone: its partner's loads repeat
            // segment sa (unconditional loads stay in flight together) and
            // the imaginary part is zero
            const int sbl = sb < a.n_seg ? sb : sa;
            const float w = a.hann[m];
            const float *xa = x + sa * hop, *xb = x + sbl * hop;
            const float re = ((xa[m] - xa[0]) - smean[sa]) * w;
            const float im = ((xb[m] - xb[0]) - smean[sbl]) * w;
            buf[e] = make_float2(re, sb < a.n_seg ? im : 0.f);
        }
        __syncthreads();
        fft_lds<kWelchThreads, kWelchBatch / 4 / kWelchThreads, false>(buf, a.log2L, np, tw);
#pragma unroll
        for (int q = 0; q < kWelchBinsPerThread; ++q) {
            const int f = tid + q * kWelchThreads;
            if (f < nb2) {
                const int fm = (L - f) & (L - 1);
                float pw = 0.f;
                for (int t = 0; t < np; ++t) {
                    const float2 Z1 = buf[(t << a.log2L) + f], Z2 = buf[(t << a.log2L) + fm];
                    pw += 0.5f * ((Z1.x * Z1.x + Z1.y * Z1.y) + (Z2.x * Z2.x + Z2.y * Z2.y));
                }
                acc[q] += pw;
            }
        }
        __syncthreads();
    }
    float *P = a.psd + g * nb2;
#pragma unroll
    for (int q = 0; q < kWelchBinsPerThread; ++q) {
        const int f = tid + q * kWelchThreads;
        if (f < nb2) P[f] = acc[q] * ((f == 0 || f == L / 2) ? a.psd_scale : 2.f * a.psd_scale);
    }
}

hipError_t launch_an_welch(const AnChunk &a, hipStream_t s)
{
    const size_t lds = sizeof(float2) * kWelchBatch;
    hipError_t e = hipFuncSetAttribute((const void *)an_welch_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(an_welch_kernel, dim3((unsigned)a.n_reg), dim3(kWelchThreads), lds, s, a);
    return hipGetLastError();
}

// -------------------------------------------------------------------- Hilbert
// One workgroup per region. The real window x (N samples) is transformed as
// the complex sequence c_m = x_2m + i x_2m+1 of length M = N/2; with
// E = (C_f + conj C_{M-f})/2 and O = (C_f - conj C_{M-f})/(2i) (the transforms
// of the even and odd samples), X_f = E + W^f O and X_{M-f} = conj(E - W^f O),
// W = exp(-2 pi i / N). The analytic weights are applied on the way (bin 0 to
// zero, bins 1..M-1 doubled, bin M kept, bins above M zero), then the inverse
// transform of length N, scaled by 1/N.
constexpr int kHilbertStageBatch = 8;   // window loads in flight per thread

template <int Q4>
__global__ __launch_bounds__(kHilbertThreads) void an_hilbert_kernel(AnChunk a)
{
    extern __shared__ float2 buf[];               // Na complex values
    __shared__ TwLds tw;
    constexpr int NT = kHilbertThreads;
    constexpr int PM = (kTwMax / 4 + 1 + NT - 1) / NT;   // bin pairs per thread
    const int tid = threadIdx.x;
    const int64_t g = blockIdx.x;
    const int N = a.Na, M = N >> 1;
    const float *x = a.xT + g * N;
    load_twiddles(tw, a.tw);
    // kHilbertStageBatch loads in flight per thread before their LDS stores
    // (indices past the window load its first pair, unused)
    for (int m0 = tid; m0 < M; m0 += kHilbertStageBatch * NT) {
        float2 v[kHilbertStageBatch];
#pragma unroll
        for (int j = 0; j < kHilbertStageBatch; ++j) {
            const int m = m0 + j * NT, mm = m < M ? m : 0;
            v[j] = make_float2(x[2 * mm], x[2 * mm + 1]);
        }
#pragma unroll
        for (int j = 0; j < kHilbertStageBatch; ++j)
            if (m0 + j * NT < M) buf[m0 + j * NT] = v[j];
    }
    __syncthreads();
    fft_lds<NT, Q4, false>(buf, a.log2Na - 1, 1, tw);
    float2 ca[PM], cb[PM];
#pragma unroll
    for (int q = 0; q < PM; ++q) {
        const int f = tid + q * NT;
        if (f <= (M >> 1)) {
            ca[q] = buf[f];
            cb[q] = buf[(M - f) & (M - 1)];
        }
    }
    __syncthreads();
    const int tstep = kTwMax >> a.log2Na;
#pragma unroll
    for (int q = 0; q < PM; ++q) {
        const int f = tid + q * NT;
        if (f <= (M >> 1)) {
            const float2 A = ca[q], B = cb[q];
            const float2 E = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));
            const float2 O = make_float2(0.5f * (A.y + B.y), -0.5f * (A.x - B.x));
            const float2 WO = cmul(twiddle(tw, f * tstep), O);
            const float2 Xf = cadd(E, WO);
            const float2 Dg = csub(E, WO);
            const float2 Xg = make_float2(Dg.x, -Dg.y);
            if (f == 0) {
                buf[0] = make_float2(0.f, 0.f);
                buf[M] = Xg;
            } else {
                buf[f] = make_float2(2.f * Xf.x, 2.f * Xf.y);
                if (M - f != f) buf[M - f] = make_float2(2.f * Xg.x, 2.f * Xg.y);
            }
        }
    }
    for (int t = M + 1 + tid; t < N; t += NT) buf[t] = make_float2(0.f, 0.f);
    __syncthreads();
    fft_lds<NT, Q4, true>(buf, a.log2Na, 1, tw);
    const float inv = 1.f / (float)N;             // a power of two: exact
    float2 *z = a.z + g * N;
    for (int t = tid; t < N; t += NT) {
        const float2 v = buf[t];
        z[t] = make_float2(v.x * inv, v.y * inv);
    }
}

template <int Q4> static hipError_t launch_hilbert_q(const AnChunk &a, hipStream_t s)
{
    const size_t lds = sizeof(float2) * (size_t)a.Na;
    hipError_t e = hipFuncSetAttribute((const void *)an_hilbert_kernel<Q4>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(an_hilbert_kernel<Q4>, dim3((unsigned)a.n_reg), dim3(kHilbertThreads), lds,
                       s, a);
    return hipGetLastError();
}

hipError_t launch_an_hilbert(const AnChunk &a, hipStream_t s)
{
    // radix-4 butterflies per thread: Na / 4 / threads, at least 1
    if (a.Na <= 4 * kHilbertThreads) return launch_hilbert_q<1>(a, s);
    if (a.Na <= 8 * kHilbertThreads) return launch_hilbert_q<2>(a, s);
    if (a.Na <= 16 * kHilbertThreads) return launch_hilbert_q<4>(a, s);
    if (a.Na <= 32 * kHilbertThreads) return launch_hilbert_q<8>(a, s);
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------ PLI
// Pairs k < l of one instance in 4 x 4 tiles of the upper triangle (tile
// (bk, bl), bk <= bl); workgroup `pass` takes tiles pass*NT .. pass*NT+NT-1,
// one per thread. The analytic signals of all regions are staged through LDS
// tc samples at a time ([k][tc + 1] layout). Each pair accumulates
// sign(Im(z_k conj z_l)) = sign(y_k x_l - x_k y_l): with z_k scaled by 2^100
// (no overflow for |z| < 1e4), clamping the scaled value to [-1, 1] gives the
// sign for every |Im| >= 2^-100 and 0 for Im = 0, so one clamp replaces two
// compares; the sum of +-1 stays exact in single precision (|sum| <= 16384).
int pli_time_chunk(int n, int Na)
{
    int tc = 64;
    while (tc > 8 && (size_t)n * (tc + 1) * sizeof(float2) > 65536) tc >>= 1;
    return tc < Na ? tc : Na;
}

int pli_passes(int n)
{
    const int nb = (n + 3) / 4;
    const int tiles = nb * (nb + 1) / 2;
    return (tiles + kPliThreads - 1) / kPliThreads;
}

constexpr int kPliStageBatch = 8;   // staging loads in flight per thread

__global__ __launch_bounds__(kPliThreads) void an_pli_kernel(AnChunk a)
{
    extern __shared__ float2 zs[];                // [n][tc + 1]
    __shared__ float red[kPliThreads / 64];
    const int tid = threadIdx.x;
    const int i = blockIdx.y, pass = blockIdx.x;
    const int n = a.n[i];
    const int nb = (n + 3) >> 2;
    const int tiles = nb * (nb + 1) / 2;
    const int u = pass * kPliThreads + tid;
    const bool active = u < tiles;                // n == 1: one tile, the diagonal only
    int bk = 0, rem = active ? u : 0;
    while (rem >= nb - bk) { rem -= nb - bk; ++bk; }   // row bk holds nb - bk tiles
    const int bl = bk + rem;
    const int tc = a.pli_tc, ld = tc + 1;
    const int64_t rb = a.rbase[i];
    const float2 *z = a.z + rb * a.Na;
    float acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = 0.f;
    const float kScale = 0x1p100f;
    const int k0 = 4 * bk, l0 = 4 * bl;
    // rows beyond n read row n-1 (their pairs are masked out below)
    int kr[4], lr[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        kr[p] = min(k0 + p, n - 1) * ld;
        lr[p] = min(l0 + p, n - 1) * ld;
    }
    // tc is a power of two: element e of a chunk is region e >> ltc, sample
    // e & (tc - 1); a thread issues kPliStageBatch loads before storing them
    // (elements past the chunk load its first one, unused)
    const int ltc = __builtin_ctz((unsigned)tc), ne = n * tc;
    for (int t0 = 0; t0 < a.Na; t0 += tc) {
        for (int e0 = tid; e0 < ne; e0 += kPliStageBatch * kPliThreads) {
            float2 v[kPliStageBatch];
#pragma unroll
            for (int j = 0; j < kPliStageBatch; ++j) {
                const int e = e0 + j * kPliThreads, ee = e < ne ? e : 0;
                v[j] = z[(int64_t)(ee >> ltc) * a.Na + t0 + (ee & (tc - 1))];
            }
#pragma unroll
            for (int j = 0; j < kPliStageBatch; ++j) {
                const int e = e0 + j * kPliThreads;
                if (e < ne) zs[(e >> ltc) * ld + (e & (tc - 1))] = v[j];
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll 4
            for (int tt = 0; tt < tc; ++tt) {
                float2 zk[4], zl[4];
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const float2 v = zs[kr[p] + tt];
                    zk[p] = make_float2(v.x * kScale, v.y * kScale);
                    zl[p] = zs[lr[p] + tt];
                }
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float im = zk[p].y * zl[q].x - zk[p].x * zl[q].y;
                        acc[p][q] += __builtin_amdgcn_fmed3f(im, -1.f, 1.f);
                    }
            }
        }
        __syncthreads();
    }
    // results of this thread's pairs
    float part = 0.f;
    const float invN = 1.f / (float)a.Na;
    if (active) {
        float *M = a.pli_out ? a.pli_out + a.pli_off[i] : nullptr;
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + p, l = l0 + q;
                if (k < n && l < n && k <= l) {
                    const float v = k < l ? fabsf(acc[p][q]) * invN : 0.f;
                    if (k < l) part += v;
                    if (M) {
                        M[(int64_t)k * n + l] = v;
                        M[(int64_t)l * n + k] = v;
                    }
                }
            }
    }
    part = wave_sum(part);
    if ((tid & 63) == 0) red[tid >> 6] = part;
    __syncthreads();
    if (tid == 0) {
        float s = 0.f;
        for (int w = 0; w < kPliThreads / 64; ++w) s += red[w];
        a.pli_part[(int64_t)i * a.pli_passes + pass] = s;
    }
}

hipError_t launch_an_pli(const AnChunk &a, int max_n, hipStream_t s)
{
    const size_t lds = (size_t)max_n * (a.pli_tc + 1) * sizeof(float2);
    hipError_t e = hipFuncSetAttribute((const void *)an_pli_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(an_pli_kernel, dim3((unsigned)a.pli_passes, (unsigned)a.n_inst),
                       dim3(kPliThreads), lds, s, a);
    return hipGetLastError();
}

// --------------------------------------------------------------------- Up/Down
// One thread per region, reading the window in the stored [t][n] layout (lanes
// of one instance read consecutive addresses) once: its min and max come from
// the Welch kernel. Thresholds are formed in single precision without
// contraction, so they equal those of any other single-precision evaluation of
// the same expressions.
constexpr int kUdUnroll = 16;

__global__ __launch_bounds__(kUdThreads) void an_ud_kernel(AnChunk a)
{
#pragma clang fp contract(off)
    const int g = blockIdx.x * kUdThreads + threadIdx.x;
    if (g >= a.n_reg) return;
    const int i = a.reg_inst[g];
    const int n = a.n[i];
    const int k = g - a.rbase[i];
    const float *x = a.samples + a.samp_off[i] + (a.n_samples - a.Na) * (int64_t)n + k;
    // the window's min and max, left in this region's slots by the Welch
    // kernel; the pass loads kUdUnroll samples before using any (more loads in
    // flight per thread; the window length is a power of two >= 16)
    int32_t *o = a.ud + (int64_t)g * 4;
    const float mn = __int_as_float(o[0]), mx = __int_as_float(o[1]);
    int su = 0, nu = 0, sd = 0, nd = 0;
    const float r = mx - mn;
    if (r >= a.ud_min_range) {
        const float half = 0.5f * r;
        const float centre = mn + half;
        const float h = a.ud_band * r;
        const float up = centre + h, dn = centre - h;
        int state = 0, entered = 0;
        bool real_entry = false;
        for (int t0 = 0; t0 < a.Na; t0 += kUdUnroll) {
            float vv[kUdUnroll];
#pragma unroll
            for (int u = 0; u < kUdUnroll; ++u) vv[u] = x[(int64_t)(t0 + u) * n];
#pragma unroll
            for (int u = 0; u < kUdUnroll; ++u) {
                const int t = t0 + u;
                const float v = vv[u];
                const int c = v > up ? 1 : (v < dn ? -1 : state);
                if (c != state) {
                    if (real_entry) {
                        if (state > 0) { su += t - entered; ++nu; }
                        else { sd += t - entered; ++nd; }
                    }
                    real_entry = state != 0;
                    state = c;
                    entered = t;
                }
            }
        }
    }
    o[0] = su;
    o[1] = nu;
    o[2] = sd;
    o[3] = nd;
}

hipError_t launch_an_ud(const AnChunk &a, hipStream_t s)
{
    hipLaunchKernelGGL(an_ud_kernel, dim3((unsigned)((a.n_reg + kUdThreads - 1) / kUdThreads)),
                       dim3(kUdThreads), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------- finalise
// One workgroup per instance: the region-mean spectrum (regions summed in
// order), its peak (lowest bin on ties), the least-squares power-law fit in
// FP64, the mean PLI, and the Up/Down sums.
__global__ __launch_bounds__(kFinalThreads) void an_final_kernel(AnChunk a)
{
    __shared__ float mean[kMaxSegment / 2 + 1];
    __shared__ float rv[kFinalThreads];
    __shared__ int ri[kFinalThreads];
    __shared__ double rd[5][kFinalThreads];
    const int tid = threadIdx.x;
    const int i = blockIdx.x;
    const int n = a.n[i];
    const int64_t rb = a.rbase[i];
    const int nb2 = a.L / 2 + 1;
    const float invn = 1.f / (float)n;
    for (int f = tid; f < nb2; f += kFinalThreads) {
        float s = 0.f;
        for (int k = 0; k < n; ++k) s += a.psd[(rb + k) * nb2 + f];
        mean[f] = s * invn;
    }
    __syncthreads();
    // peak over bins 1..L/2
    float best = -1.f;
    int bi = 0x7fffffff;
    for (int f = 1 + tid; f < nb2; f += kFinalThreads) {
        const float v = mean[f];
        if (v > best) { best = v; bi = f; }
    }
    // fit sums
    double c = 0.0, sx = 0.0, sy = 0.0, sxx = 0.0, sxy = 0.0;
    for (int f = 1 + tid; f < nb2; f += kFinalThreads) {
        const double fr = (double)f * a.df_hz;
        const float v = mean[f];
        if (fr >= a.fit_lo && fr <= a.fit_hi && v > 0.f) {
            const double X = log10(fr), Y = log10((double)v);
            c += 1.0; sx += X; sy += Y; sxx += X * X; sxy += X * Y;
        }
    }
    rv[tid] = best;
    ri[tid] = bi;
    rd[0][tid] = c; rd[1][tid] = sx; rd[2][tid] = sy; rd[3][tid] = sxx; rd[4][tid] = sxy;
    __syncthreads();
    for (int w = kFinalThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
            const float v2 = rv[tid + w];
            const int i2 = ri[tid + w];
            if (v2 > rv[tid] || (v2 == rv[tid] && i2 < ri[tid])) { rv[tid] = v2; ri[tid] = i2; }
            for (int m = 0; m < 5; ++m) rd[m][tid] += rd[m][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        vadx_analysis r;
        r.psd_peak_bin = ri[0];
        r.psd_fmax_hz = (float)((double)ri[0] * a.df_hz);
        r.psd_ampmax = rv[0];
        const double cn = rd[0][0], Sx = rd[1][0], Sy = rd[2][0], Sxx = rd[3][0], Sxy = rd[4][0];
        if (cn >= 2.0) {
            const double slope = (cn * Sxy - Sx * Sy) / (cn * Sxx - Sx * Sx);
            r.psd_slope_a = (float)(-slope);
            r.psd_log10_b = (float)((Sy - slope * Sx) / cn);
            r.psd_fit_bins = (int32_t)cn;
        } else {
            r.psd_slope_a = 0.f;
            r.psd_log10_b = 0.f;
            r.psd_fit_bins = 0;
        }
        float ps = 0.f;
        for (int p = 0; p < a.pli_passes; ++p) ps += a.pli_part[(int64_t)i * a.pli_passes + p];
        r.mean_pli = n > 1 ? ps / (0.5f * (float)n * (float)(n - 1)) : 0.f;
        int64_t su = 0, sd = 0;
        int32_t nu = 0, nd = 0;
        for (int k = 0; k < n; ++k) {
            const int32_t *u = a.ud + (rb + k) * 4;
            su += u[0]; nu += u[1]; sd += u[2]; nd += u[3];
        }
        r.ud_up_samples = su;
        r.ud_down_samples = sd;
        r.ud_up_count = nu;
        r.ud_down_count = nd;
        r.ud_up_ms = nu ? (float)((double)su * a.period_ms / nu) : 0.f;
        r.ud_down_ms = nd ? (float)((double)sd * a.period_ms / nd) : 0.f;
        r.reserved = 0.f;
        a.out[i] = r;
    }
}

hipError_t launch_an_final(const AnChunk &a, hipStream_t s)
{
    hipLaunchKernelGGL(an_final_kernel, dim3((unsigned)a.n_inst), dim3(kFinalThreads), 0, s, a);
    return hipGetLastError();
}

} // namespace vadx
