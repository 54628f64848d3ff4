// analysis_api.cpp -- host side of the analysis metrics (Section 2.6,
// Table 2): argument checks, workspace layout, passes over whole instances and
// the launch sequence (transpose, Welch spectra, analytic signals, phase lag
// index, Up/Down durations, per-instance reduction).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "analysis_engine.h"
#include "vadx.h"

namespace vadx {

namespace {

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

bool pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2(int64_t x)
{
    int r = 0;
    while ((int64_t(1) << (r + 1)) <= x) ++r;
    return r;
}

struct Resolved {
    int Na = 0, L = 0, n_seg = 0, nb2 = 0;
};

vadx_status resolve(int64_t n_samples, const vadx_analysis_cfg *cfg, Resolved *r, std::string &err)
{
    if (!cfg) { err = "null analysis settings"; return VADX_E_ARG; }
    if (n_samples < kMinSegment) { err = "fewer than 16 samples"; return VADX_E_ARG; }
    int64_t Na = cfg->window;
    if (Na == 0) {
        Na = int64_t(1) << ilog2(n_samples);
        Na = std::min<int64_t>(Na, kTwMax);
    }
    if (!pow2(Na) || Na > n_samples || Na < kMinSegment) {
        err = "window must be a power of two in [16, sample count]";
        return VADX_E_ARG;
    }
    if (Na > kTwMax) { err = "window longer than 16384 samples"; return VADX_E_UNSUPPORTED; }
    int64_t L = cfg->segment ? cfg->segment : std::min<int64_t>(1024, Na);
    if (!pow2(L) || L < kMinSegment || L > Na || L > kMaxSegment) {
        err = "segment must be a power of two in [16, min(window, 8192)]";
        return VADX_E_ARG;
    }
    if (!(std::isfinite(cfg->fit_lo_hz) && std::isfinite(cfg->fit_hi_hz) &&
          cfg->fit_lo_hz <= cfg->fit_hi_hz)) {
        err = "invalid fit band";
        return VADX_E_ARG;
    }
    if (!(std::isfinite(cfg->ud_band) && cfg->ud_band >= 0.f && std::isfinite(cfg->ud_min_range_khz) &&
          cfg->ud_min_range_khz >= 0.f)) {
        err = "invalid Up/Down settings";
        return VADX_E_ARG;
    }
    r->Na = (int)Na;
    r->L = (int)L;
    r->n_seg = (int)((Na - L) / (L / 2) + 1);
    r->nb2 = (int)(L / 2 + 1);
    return VADX_OK;
}

// Bytes per region of one pass and the fixed part (twiddles, window, padding).
void layout_sizes(const Resolved &r, int n_max, size_t *per_region, size_t *fixed)
{
    const int P = pli_passes(std::max(n_max, 1));
    *per_region = 8 + 4 + 4 + 4 + 8                  // instance tables (at most one instance per region)
                  + (size_t)r.Na * 4 + (size_t)r.Na * 8 // window rows, analytic signals
                  + (size_t)r.nb2 * 4 + 16              // spectra, Up/Down sums
                  + (size_t)P * 4;                      // PLI partial sums
    *fixed = sizeof(float2) * kTwMax + (size_t)r.L * 4 + 16 * 256;
}

} // namespace

vadx_status analysis_bytes(int64_t n_samples, int32_t n_max, int64_t regions_per_pass,
                           const vadx_analysis_cfg *cfg, size_t *bytes, std::string &err)
{
    if (!bytes) { err = "null argument"; return VADX_E_ARG; }
    if (n_max < 1 || n_max > 512) { err = "region count must be in [1, 512]"; return VADX_E_ARG; }
    if (regions_per_pass < n_max) { err = "a pass must hold one instance"; return VADX_E_ARG; }
    Resolved r;
    vadx_status st = resolve(n_samples, cfg, &r, err);
    if (st) return st;
    size_t per = 0, fixed = 0;
    layout_sizes(r, n_max, &per, &fixed);
    *bytes = fixed + per * (size_t)regions_per_pass;
    return VADX_OK;
}

#define AN_TRY(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            err = std::string(#expr) + ": " + hipGetErrorString(e_);                   \
            return VADX_E_HIP;                                                         \
        }                                                                              \
    } while (0)

vadx_status run_analysis(int device, hipStream_t stream, const AnInstances &in, double period_ms,
                         const vadx_analysis_cfg *cfg, void *ws, size_t ws_bytes,
                         vadx_analysis *out, float *psd_out, float *pli_out, AnTimer *timer,
                         std::string &err)
{
    if (!ws || ((uintptr_t)ws & 255u) || !out || !in.samples) {
        err = "null or misaligned pointer";
        return VADX_E_ARG;
    }
    if (!(period_ms > 0.0) || !std::isfinite(period_ms)) { err = "invalid sample period"; return VADX_E_ARG; }
    if (in.n_inst < 0) { err = "negative instance count"; return VADX_E_ARG; }
    Resolved r;
    vadx_status st = resolve(in.n_samples, cfg, &r, err);
    if (st) return st;
    if (in.n_inst == 0) return VADX_OK;
    int n_max = 0;
    for (int64_t i = 0; i < in.n_inst; ++i) {
        if (in.n[i] < 1 || in.n[i] > 512) { err = "region count must be in [1, 512]"; return VADX_E_ARG; }
        n_max = std::max(n_max, (int)in.n[i]);
    }
    size_t per = 0, fixed = 0;
    layout_sizes(r, n_max, &per, &fixed);
    if (ws_bytes < fixed + per * (size_t)n_max) {
        err = "analysis workspace too small for one instance";
        return VADX_E_OOM;
    }
    const int64_t R_cap = (int64_t)((ws_bytes - fixed) / per);
    const int P = pli_passes(n_max);

    // workspace sections
    char *base = (char *)ws;
    size_t off = 0;
    auto take = [&](size_t bytes) { char *p = base + off; off = up256(off + bytes); return p; };
    float2 *d_tw = (float2 *)take(sizeof(float2) * kTwMax);
    float *d_hann = (float *)take(sizeof(float) * r.L);
    int64_t *d_samp = (int64_t *)take(8 * (size_t)R_cap);
    int32_t *d_n = (int32_t *)take(4 * (size_t)R_cap);
    int32_t *d_rbase = (int32_t *)take(4 * (size_t)R_cap);
    int32_t *d_reg = (int32_t *)take(4 * (size_t)R_cap);
    int64_t *d_pli_off = (int64_t *)take(8 * (size_t)R_cap);
    float *d_xT = (float *)take(4 * (size_t)R_cap * r.Na);
    float2 *d_z = (float2 *)take(8 * (size_t)R_cap * r.Na);
    float *d_psd = (float *)take(4 * (size_t)R_cap * r.nb2);
    int32_t *d_ud = (int32_t *)take(16 * (size_t)R_cap);
    float *d_part = (float *)take(4 * (size_t)R_cap * P);
    if (off > ws_bytes) { err = "analysis workspace layout overflow"; return VADX_E_OOM; }

    AN_TRY(hipSetDevice(device));
    std::vector<float2> tw(kTwMax);
    for (int j = 0; j < kTwMax; ++j) {
        const double ang = 2.0 * M_PI * (double)j / (double)kTwMax;
        tw[j] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
    }
    std::vector<float> hann(r.L);
    double sw2 = 0.0;
    for (int m = 0; m < r.L; ++m) {
        const double w = 0.5 - 0.5 * std::cos(2.0 * M_PI * (double)m / (double)r.L);
        hann[m] = (float)w;
        sw2 += w * w;
    }
    AN_TRY(hipMemcpyAsync(d_tw, tw.data(), sizeof(float2) * kTwMax, hipMemcpyHostToDevice, stream));
    AN_TRY(hipMemcpyAsync(d_hann, hann.data(), sizeof(float) * r.L, hipMemcpyHostToDevice, stream));

    const double fs = 1000.0 / period_ms;
    AnChunk a{};
    a.samples = in.samples;
    a.samp_off = d_samp;
    a.n = d_n;
    a.rbase = d_rbase;
    a.reg_inst = d_reg;
    a.pli_off = d_pli_off;
    a.n_samples = in.n_samples;
    a.Na = r.Na;
    a.log2Na = ilog2(r.Na);
    a.L = r.L;
    a.log2L = ilog2(r.L);
    a.n_seg = r.n_seg;
    a.psd_scale = (float)(1e6 / (fs * sw2 * (double)r.n_seg));
    a.ud_band = cfg->ud_band;
    a.ud_min_range = cfg->ud_min_range_khz;
    a.df_hz = fs / (double)r.L;
    a.fit_lo = cfg->fit_lo_hz;
    a.fit_hi = cfg->fit_hi_hz;
    a.period_ms = period_ms;
    a.tw = d_tw;
    a.hann = d_hann;
    a.xT = d_xT;
    a.z = d_z;
    a.psd = d_psd;
    a.ud = d_ud;
    a.pli_part = d_part;
    a.pli_out = pli_out;

    // Host tables of every pass, built before the first copy: each pass copies
    // its own slice, which nothing modifies afterwards (pageable host copies are
    // staged when the call returns).
    std::vector<int64_t> h_pli(in.n_inst), chunk_first;
    std::vector<int32_t> h_rbase(in.n_inst), h_reg;
    h_reg.reserve(4096);
    int64_t po = 0;
    for (int64_t i0 = 0; i0 < in.n_inst;) {
        chunk_first.push_back(i0);
        int64_t i1 = i0, regs = 0;
        // (instances per pass also bounded by the grid's y extent)
        while (i1 < in.n_inst && regs + in.n[i1] <= R_cap && i1 - i0 < 65535) {
            h_rbase[i1] = (int32_t)regs;
            h_pli[i1] = po;
            po += (int64_t)in.n[i1] * in.n[i1];
            for (int k = 0; k < in.n[i1]; ++k) h_reg.push_back((int32_t)(i1 - i0));
            regs += in.n[i1];
            ++i1;
        }
        i0 = i1;
    }
    chunk_first.push_back(in.n_inst);
    int64_t reg_done = 0;
    for (size_t c = 0; c + 1 < chunk_first.size(); ++c) {
        const int64_t i0 = chunk_first[c], i1 = chunk_first[c + 1], ni = i1 - i0;
        int64_t regs = 0;
        int cmax = 0;
        for (int64_t i = i0; i < i1; ++i) {
            regs += in.n[i];
            cmax = std::max(cmax, (int)in.n[i]);
        }
        AN_TRY(hipMemcpyAsync(d_samp, in.samp_off + i0, 8 * ni, hipMemcpyHostToDevice, stream));
        AN_TRY(hipMemcpyAsync(d_n, in.n + i0, 4 * ni, hipMemcpyHostToDevice, stream));
        AN_TRY(hipMemcpyAsync(d_rbase, h_rbase.data() + i0, 4 * ni, hipMemcpyHostToDevice, stream));
        AN_TRY(hipMemcpyAsync(d_reg, h_reg.data() + reg_done, 4 * regs, hipMemcpyHostToDevice, stream));
        AN_TRY(hipMemcpyAsync(d_pli_off, h_pli.data() + i0, 8 * ni, hipMemcpyHostToDevice, stream));
        a.n_inst = (int32_t)ni;
        a.n_reg = (int32_t)regs;
        a.pli_passes = pli_passes(cmax);
        a.pli_tc = pli_time_chunk(cmax, r.Na);
        a.out = out + i0;
        for (int kk = 0; kk < kAnKernels; ++kk) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timer) {
                AN_TRY(hipEventCreate(&e0));
                AN_TRY(hipEventCreate(&e1));
                timer->ev[kk].emplace_back(e0, e1);
                AN_TRY(hipEventRecord(e0, stream));
            }
            switch (kk) {
            case 0: AN_TRY(launch_an_transpose(a, cmax, stream)); break;
            case 1: AN_TRY(launch_an_welch(a, stream)); break;
            case 2: AN_TRY(launch_an_hilbert(a, stream)); break;
            case 3: AN_TRY(launch_an_pli(a, cmax, stream)); break;
            case 4: AN_TRY(launch_an_ud(a, stream)); break;
            default: AN_TRY(launch_an_final(a, stream)); break;
            }
            if (timer) AN_TRY(hipEventRecord(e1, stream));
        }
        if (psd_out)
            AN_TRY(hipMemcpyAsync(psd_out + reg_done * r.nb2, d_psd, sizeof(float) * regs * r.nb2,
                                  hipMemcpyDeviceToDevice, stream));
        reg_done += regs;
    }
    return VADX_OK;
}

} // namespace vadx

extern "C" vadx_status vadx_analysis_defaults(vadx_analysis_cfg *out)
{
    if (!out) return VADX_E_ARG;
    out->window = 0;
    out->segment = 0;
    out->fit_lo_hz = 1.0;
    out->fit_hi_hz = 100.0;
    out->ud_band = 0.1f;
    out->ud_min_range_khz = 1e-3f;
    return VADX_OK;
}

extern "C" vadx_status vadx_analysis_ws_bytes(int64_t n_samples, int32_t n_max,
                                              int64_t regions_per_pass,
                                              const vadx_analysis_cfg *cfg, size_t *bytes)
{
    std::string err;
    return vadx::analysis_bytes(n_samples, n_max, regions_per_pass, cfg, bytes, err);
}
