// mlp_api.cpp -- host side of the surrogate-network entry points of vadx.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mlp_engine.h"
#include "vadx.h"

using namespace vadx;

struct vadx_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    vadx_mlp_cfg cfg{};
    MlpArgs a{};
    float *dev = nullptr;            // params | m | v | grad
    float *partial = nullptr;        // per-tile gradient slots
    int partial_tiles = 0;
    float *losses = nullptr;         // per-step loss sums
    int64_t losses_n = 0;
    int64_t step = 0;                // Adam steps taken
    double *stat = nullptr;          // target statistics scratch (12 doubles)
    float *loss1 = nullptr;          // loss sum of one gradient evaluation
    // selection scratch: 256 histogram bins, then per-tile counts and bases
    vadx::SelScratch sel;
};

static vadx_status mfail(vadx_mlp *m, vadx_status st, const char *msg, hipError_t e = hipSuccess)
{
    if (m) {
        m->err = msg;
        if (e != hipSuccess) m->err += std::string(": ") + hipGetErrorString(e);
    }
    return st;
}

#define MHIP(m, expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return mfail((m), e_ == hipErrorOutOfMemory ? VADX_E_OOM : VADX_E_HIP, #expr, e_); \
    } while (0)

static hipError_t ensure_partial(vadx_mlp *m, int tiles)
{
    if (tiles <= m->partial_tiles) return hipSuccess;
    if (m->partial) (void)hipFree(m->partial);
    m->partial = nullptr;
    m->partial_tiles = 0;
    hipError_t e = hipMalloc((void **)&m->partial, (size_t)tiles * kMlpSlot * sizeof(float));
    if (e == hipSuccess) m->partial_tiles = tiles;
    m->a.partial = m->partial;
    return e;
}

// Target mean and population standard deviation per output column (FP64).
__global__ void mlp_target_stats_kernel(const float *Y, int64_t n, double *out)
{
    __shared__ double s1[256], s2[256];
    const int c = blockIdx.x, tid = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t i = tid; i < n; i += 256) {
        const double y = Y[i * 6 + c];
        a += y;
        b += y * y;
    }
    s1[tid] = a;
    s2[tid] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) { s1[tid] += s1[tid + s]; s2[tid] += s2[tid + s]; }
        __syncthreads();
    }
    if (tid == 0) {
        const double mean = n > 0 ? s1[0] / (double)n : 0.0;
        const double var = n > 0 ? s2[0] / (double)n - mean * mean : 0.0;
        out[c] = mean;
        out[6 + c] = var > 0.0 ? std::sqrt(var) : 1.0;
    }
}

namespace vadx {

#define SHIP(expr)                                                                     \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            err = std::string(#expr) + ": " + hipGetErrorString(e_);                   \
            return e_ == hipErrorOutOfMemory ? VADX_E_OOM : VADX_E_HIP;                \
        }                                                                              \
    } while (0)

size_t select_scratch_bytes(int64_t tiles)
{
    const size_t off_cnt = 256 * sizeof(uint32_t);
    const size_t off_eq = (off_cnt + tiles * sizeof(uint32_t) + 255) & ~(size_t)255;
    return off_eq + 2 * tiles * sizeof(int64_t);
}

vadx_status select_run(hipStream_t s, SelScratch &sc, const float *score, int64_t n, int64_t k,
                       float audit_frac, uint32_t seed, int64_t *sel, uint8_t *is_audit,
                       int64_t capacity, int64_t *n_sel, std::string &err,
                       uint32_t *host_counts, int64_t *host_bases)
{
    if (!n_sel || n < 0 || k < 0 || (n > 0 && !score) || capacity < 0 ||
        (capacity > 0 && !sel) || !(audit_frac >= 0.f && audit_frac <= 1.f)) {
        err = "bad arguments";
        return VADX_E_ARG;
    }
    if (n > ((int64_t)1 << 40)) { err = "too many points"; return VADX_E_UNSUPPORTED; }
    *n_sel = 0;
    if (n == 0) return VADX_OK;
    if (k > n) k = n;
    const int64_t tiles = select_tiles(n);
    // scratch layout: hist u32[256] | counts u32[tiles] | eq_base i64[tiles] | sel_base i64[tiles]
    const size_t off_cnt = 256 * sizeof(uint32_t);
    const size_t off_eq = (off_cnt + tiles * sizeof(uint32_t) + 255) & ~(size_t)255;
    const size_t off_sb = off_eq + tiles * sizeof(int64_t);
    const size_t bytes = select_scratch_bytes(tiles);
    if (tiles > sc.tiles) {
        if (sc.p) (void)hipFree(sc.p);
        sc.p = nullptr;
        sc.tiles = -1;
        SHIP(hipMalloc(&sc.p, bytes));
        sc.tiles = tiles;
    }
    char *base = (char *)sc.p;
    uint32_t *hist = (uint32_t *)base;
    uint32_t *counts = (uint32_t *)(base + off_cnt);
    int64_t *eq_base = (int64_t *)(base + off_eq);
    int64_t *sel_base = (int64_t *)(base + off_sb);

    // radix select of the k-th largest key: T and the number of keys equal to
    // T that belong to the top k
    uint32_t prefix = 0, mask = 0;
    int64_t need = k;
    const int use_top = k > 0;
    if (use_top) {
        for (int shift = 24; shift >= 0; shift -= 8) {
            uint32_t h[256];
            SHIP(hipMemsetAsync(hist, 0, 256 * sizeof(uint32_t), s));
            SHIP(launch_sel_hist(score, n, prefix, mask, shift, hist, s));
            SHIP(hipMemcpyAsync(h, hist, sizeof(h), hipMemcpyDeviceToHost, s));
            SHIP(hipStreamSynchronize(s));
            int b = 255;
            for (; b > 0; --b) {
                if ((int64_t)h[b] >= need) break;
                need -= h[b];
            }
            prefix |= (uint32_t)b << shift;
            mask |= 0xFFu << shift;
        }
    }
    std::vector<uint32_t> hc_own;
    std::vector<int64_t> hb_own;
    if (!host_counts || !host_bases) {
        hc_own.resize((size_t)tiles);
        hb_own.resize((size_t)tiles);
    }
    uint32_t *hc = host_counts ? host_counts : hc_own.data();
    int64_t *hb = host_bases ? host_bases : hb_own.data();
    // phase 0: keys equal to T per tile -> eq_base
    if (use_top) {
        SHIP(launch_sel_compact(score, n, 0, 1, prefix, need, 0.f, seed, nullptr, nullptr,
                                counts, nullptr, nullptr, s));
        SHIP(hipMemcpyAsync(hc, counts, tiles * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        SHIP(hipStreamSynchronize(s));
    }
    int64_t acc = 0;
    for (int64_t t = 0; t < tiles; ++t) {
        hb[t] = acc;
        acc += use_top ? hc[t] : 0;
    }
    SHIP(hipMemcpyAsync(eq_base, hb, tiles * sizeof(int64_t), hipMemcpyHostToDevice, s));
    // phase 1: selected points per tile -> sel_base
    SHIP(launch_sel_compact(score, n, 1, use_top, prefix, need, audit_frac, seed, eq_base,
                            nullptr, counts, nullptr, nullptr, s));
    SHIP(hipMemcpyAsync(hc, counts, tiles * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SHIP(hipStreamSynchronize(s));
    acc = 0;
    for (int64_t t = 0; t < tiles; ++t) {
        hb[t] = acc;
        acc += hc[t];
    }
    *n_sel = acc;
    if (acc > capacity) { err = "selection larger than the output capacity"; return VADX_E_OOM; }
    SHIP(hipMemcpyAsync(sel_base, hb, tiles * sizeof(int64_t), hipMemcpyHostToDevice, s));
    // phase 2: write the indices
    SHIP(launch_sel_compact(score, n, 2, use_top, prefix, need, audit_frac, seed, eq_base,
                            sel_base, nullptr, sel, is_audit, s));
    SHIP(hipStreamSynchronize(s));
    return VADX_OK;
}

} // namespace vadx

extern "C" {

vadx_status vadx_mlp_create(vadx_ctx *ctx, const vadx_mlp_cfg *cfg, const float *init_params,
                            vadx_mlp **out)
{
    (void)ctx;
    if (!cfg || !init_params || !out) return VADX_E_ARG;
    *out = nullptr;
    for (int i = 0; i < 4; ++i)
        if (!(cfg->x_hi[i] > cfg->x_lo[i])) return VADX_E_ARG;
    if (!(cfg->lr > 0 && cfg->beta1 >= 0 && cfg->beta1 < 1 && cfg->beta2 >= 0 && cfg->beta2 < 1 &&
          cfg->eps > 0))
        return VADX_E_ARG;
    for (int i = 0; i < kMlpParams; ++i)
        if (!std::isfinite(init_params[i])) return VADX_E_ARG;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return VADX_E_HIP;
    vadx_mlp *m = new vadx_mlp();
    m->device = device;
    m->stream = (hipStream_t)cfg->hip_stream;
    m->cfg = *cfg;
    if (hipMalloc((void **)&m->dev, sizeof(float) * 4 * kMlpParams) != hipSuccess ||
        hipMalloc((void **)&m->stat, sizeof(double) * 12) != hipSuccess ||
        hipMalloc((void **)&m->loss1, sizeof(float)) != hipSuccess) {
        vadx_mlp_destroy(m);
        return VADX_E_OOM;
    }
    MlpArgs &a = m->a;
    a.params = m->dev;
    a.m = m->dev + kMlpParams;
    a.v = m->dev + 2 * kMlpParams;
    a.grad = m->dev + 3 * kMlpParams;
    for (int i = 0; i < 4; ++i) {
        a.x_lo[i] = cfg->x_lo[i];
        a.x_scale[i] = 2.0f / (cfg->x_hi[i] - cfg->x_lo[i]);
    }
    for (int i = 0; i < 6; ++i) {
        a.y_mean[i] = 0.f;
        a.y_std[i] = 1.f;
        a.y_rstd[i] = 1.f;
    }
    a.lr = cfg->lr;
    a.beta1 = cfg->beta1;
    a.beta2 = cfg->beta2;
    a.eps = cfg->eps;
    a.score_out0 = 0;
    a.score_out1 = 5;
    if (hipMemcpyAsync(a.params, init_params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice,
                       m->stream) != hipSuccess ||
        hipMemsetAsync(a.m, 0, sizeof(float) * 2 * kMlpParams, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess) {
        vadx_mlp_destroy(m);
        return VADX_E_HIP;
    }
    *out = m;
    return VADX_OK;
}

void vadx_mlp_destroy(vadx_mlp *m)
{
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    if (m->dev) (void)hipFree(m->dev);
    if (m->partial) (void)hipFree(m->partial);
    if (m->losses) (void)hipFree(m->losses);
    if (m->stat) (void)hipFree(m->stat);
    if (m->loss1) (void)hipFree(m->loss1);
    if (m->sel.p) (void)hipFree(m->sel.p);
    delete m;
}

const char *vadx_mlp_last_error(const vadx_mlp *m) { return m ? m->err.c_str() : "null network"; }

vadx_status vadx_mlp_fit_target_norm(vadx_mlp *m, const float *Y, int64_t n)
{
    if (!m || !Y || n <= 0) return mfail(m, VADX_E_ARG, "bad target array");
    hipLaunchKernelGGL(mlp_target_stats_kernel, dim3(6), dim3(256), 0, m->stream, Y, n, m->stat);
    MHIP(m, hipGetLastError());
    double h[12];
    MHIP(m, hipMemcpyAsync(h, m->stat, sizeof(h), hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    for (int i = 0; i < 6; ++i) {
        m->a.y_mean[i] = (float)h[i];
        m->a.y_std[i] = (float)h[6 + i];
        m->a.y_rstd[i] = (float)(1.0 / h[6 + i]);
    }
    return VADX_OK;
}

vadx_status vadx_mlp_get_target_norm(vadx_mlp *m, float *mean, float *std_)
{
    if (!m || !mean || !std_) return VADX_E_ARG;
    for (int i = 0; i < 6; ++i) { mean[i] = m->a.y_mean[i]; std_[i] = m->a.y_std[i]; }
    return VADX_OK;
}

vadx_status vadx_mlp_set_target_norm(vadx_mlp *m, const float *mean, const float *std_)
{
    if (!m || !mean || !std_) return VADX_E_ARG;
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(mean[i]) || !(std_[i] > 0.f)) return mfail(m, VADX_E_ARG, "bad normalisation");
    for (int i = 0; i < 6; ++i) {
        m->a.y_mean[i] = mean[i];
        m->a.y_std[i] = std_[i];
        m->a.y_rstd[i] = 1.0f / std_[i];
    }
    return VADX_OK;
}

vadx_status vadx_mlp_get_params(vadx_mlp *m, float *out)
{
    if (!m || !out) return VADX_E_ARG;
    MHIP(m, hipMemcpyAsync(out, m->a.params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    return VADX_OK;
}

vadx_status vadx_mlp_set_params(vadx_mlp *m, const float *p)
{
    if (!m || !p) return VADX_E_ARG;
    MHIP(m, hipMemcpyAsync(m->a.params, p, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    return VADX_OK;
}

// Loss and gradient over n samples (device arrays) without an update.
vadx_status vadx_mlp_grad(vadx_mlp *m, const float *X, const float *Y, int64_t n, float *grad_out,
                          float *loss_out)
{
    if (!m || !X || !Y || n <= 0 || n > (1 << 24) || !grad_out || !loss_out)
        return mfail(m, VADX_E_ARG, "bad arguments");
    const int tiles = (int)((n + kMlpTile - 1) / kMlpTile);
    MHIP(m, ensure_partial(m, tiles));
    MlpArgs a = m->a;
    a.loss_out = m->loss1;
    hipError_t e = launch_mlp_grad(a, X, Y, (int)n, (int)n, m->stream);
    if (e == hipSuccess) e = launch_mlp_adam(a, tiles, 1.f, 1.f, 0, 0, m->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(grad_out, a.grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, m->stream);
    float l = 0.f;
    if (e == hipSuccess) e = hipMemcpyAsync(&l, m->loss1, sizeof(float), hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return mfail(m, VADX_E_HIP, "gradient", e);
    *loss_out = l / (6.0f * (float)n);
    return VADX_OK;
}

vadx_status vadx_mlp_train(vadx_mlp *m, const float *X, const float *Y, int64_t n, int32_t epochs,
                           int32_t batch, float *loss_hist)
{
    if (!m || !X || !Y || n <= 0 || epochs < 0 || batch <= 0 || batch > (1 << 20) || !loss_hist)
        return mfail(m, VADX_E_ARG, "bad arguments");
    const int64_t per_epoch = (n + batch - 1) / batch;
    const int64_t total = per_epoch * epochs;
    if (total > m->losses_n) {
        if (m->losses) (void)hipFree(m->losses);
        m->losses = nullptr;
        m->losses_n = 0;
        MHIP(m, hipMalloc((void **)&m->losses, sizeof(float) * std::max<int64_t>(total, 1)));
        m->losses_n = total;
    }
    MHIP(m, ensure_partial(m, (batch + kMlpTile - 1) / kMlpTile));
    MlpArgs a = m->a;
    a.loss_out = m->losses;
    int64_t k = 0;
    for (int ep = 0; ep < epochs; ++ep)
        for (int64_t b0 = 0; b0 < n; b0 += batch, ++k) {
            const int nb = (int)std::min<int64_t>(batch, n - b0);
            const int tiles = (nb + kMlpTile - 1) / kMlpTile;
            const int64_t t = ++m->step;
            const float c1 = (float)(1.0 / (1.0 - std::pow((double)a.beta1, (double)t)));
            const float c2 = (float)(1.0 / (1.0 - std::pow((double)a.beta2, (double)t)));
            MHIP(m, launch_mlp_grad(a, X + b0 * 4, Y + b0 * 6, nb, nb, m->stream));
            MHIP(m, launch_mlp_adam(a, tiles, c1, c2, 1, (int)k, m->stream));
        }
    std::vector<float> h((size_t)std::max<int64_t>(total, 1));
    if (total > 0)
        MHIP(m, hipMemcpyAsync(h.data(), m->losses, sizeof(float) * total, hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    for (int ep = 0; ep < epochs; ++ep) {
        double s = 0.0;
        for (int64_t q = 0; q < per_epoch; ++q) s += h[ep * per_epoch + q];
        loss_hist[ep] = (float)(s / (6.0 * (double)n));
    }
    return VADX_OK;
}

vadx_status vadx_mlp_predict(vadx_mlp *m, const float *X, int64_t n, float *Y, float *J,
                             float *score, int32_t score_out0, int32_t score_out1)
{
    if (!m || n < 0 || (n > 0 && (!X || !Y)) || score_out0 < 0 || score_out0 > 5 ||
        score_out1 < 0 || score_out1 > 5)
        return mfail(m, VADX_E_ARG, "bad arguments");
    MlpArgs a = m->a;
    a.score_out0 = score_out0;
    a.score_out1 = score_out1;
    MHIP(m, launch_mlp_predict(a, X, n, Y, J, score, m->stream));
    return VADX_OK;
}

vadx_status vadx_mlp_select(vadx_mlp *m, const float *score, int64_t n, int64_t k,
                            float audit_frac, uint32_t seed, int64_t *sel, uint8_t *is_audit,
                            int64_t capacity, int64_t *n_sel)
{
    if (!m) return VADX_E_ARG;
    std::string err;
    vadx_status st = select_run(m->stream, m->sel, score, n, k, audit_frac, seed, sel, is_audit,
                                capacity, n_sel, err);
    if (st) return mfail(m, st, err.c_str());
    return VADX_OK;
}

} // extern "C"
