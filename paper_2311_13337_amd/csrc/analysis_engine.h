// analysis_engine.h -- device-side layout and launchers of the analysis
// metrics (Section 2.6, Table 2): Welch power spectra, analytic signals and
// the phase lag index, Up/Down state durations, per-instance reduction.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <utility>
#include <vector>

#include "vadx.h"

namespace vadx {

// Largest FFT length (analysis window); the twiddle table holds
// exp(-2 pi i j / kTwMax), j < kTwMax, which serves every power-of-two length
// up to it.
constexpr int kTwMax = 16384;
// Welch segments are transformed kWelchBatch complex values at a time (LDS).
constexpr int kWelchBatch = 8192;
constexpr int kWelchThreads = 512;
constexpr int kHilbertThreads = 512;
constexpr int kPliThreads = 256;
constexpr int kUdThreads = 256;
constexpr int kFinalThreads = 256;
constexpr int kMinSegment = 16;
constexpr int kMaxSegment = 8192;

// One pass over a chunk of instances. Region g of the chunk (0 <= g < R) is
// region g - rbase[i] of chunk instance i = reg_inst[g]; per-region buffers are
// indexed by g.
struct AnChunk {
    const float *samples;        // base of the stored samples
    const int64_t *samp_off;     // [I] floats: instance's [n_samples][n] block
    const int32_t *n;            // [I] regions
    const int32_t *rbase;        // [I] first chunk region of the instance
    const int32_t *reg_inst;     // [R] chunk instance of each region
    const int64_t *pli_off;      // [I] floats into pli_out (when given)
    int32_t n_inst, n_reg;
    int64_t n_samples;           // per instance (the window is the last Na)
    int32_t Na, log2Na;          // analysis window
    int32_t L, log2L;            // Welch segment
    int32_t n_seg;               // Welch segments per region
    int32_t pli_passes;          // PLI workgroups per instance
    int32_t pli_tc;              // PLI samples staged per chunk of time
    float psd_scale;             // 1e6 / (fs sum w^2 n_seg): kHz^2 -> Hz^2/Hz
    float ud_band, ud_min_range;
    double df_hz, fit_lo, fit_hi, period_ms;
    const float2 *tw;            // [kTwMax]
    const float *hann;           // [L]
    float *xT;                   // [R][Na] window, time-contiguous
    float2 *z;                   // [R][Na] analytic signals
    float *psd;                  // [R][L/2+1]
    int32_t *ud;                 // [R][4] Up sum, Up count, Down sum, Down count (slots 0, 1 carry
                                 // the window's min, max as float bits from Welch to Up/Down)
    float *pli_part;             // [I][pli_passes] sums of PLI over a workgroup's pairs
    float *pli_out;              // nullable
    vadx_analysis *out;          // [I] results of this chunk's instances
};

hipError_t launch_an_transpose(const AnChunk &a, int max_n, hipStream_t s);
hipError_t launch_an_welch(const AnChunk &a, hipStream_t s);
hipError_t launch_an_hilbert(const AnChunk &a, hipStream_t s);
hipError_t launch_an_pli(const AnChunk &a, int max_n, hipStream_t s);
hipError_t launch_an_ud(const AnChunk &a, hipStream_t s);
hipError_t launch_an_final(const AnChunk &a, hipStream_t s);

// Samples staged per PLI time chunk for n regions and the workgroups per
// instance.
int pli_time_chunk(int n, int Na);
int pli_passes(int n);

// BOLD (bold.hip): one thread per region of the instances described by the
// tables; out_off[i] = floats to instance i's [n_tr][n] output block; emit[m]
// = the sample count after which BOLD sample m is taken.
struct BoldArgs {
    const float *samples;
    const int64_t *samp_off;
    const int32_t *n;
    const int32_t *rbase;
    const int32_t *reg_inst;
    const int64_t *out_off;
    const int32_t *emit;
    int64_t n_reg, n_samples;
    int32_t n_tr;
    float kappa, gamma, inv_tau0, inv_alpha, inv_E0, l2_1mE0;
    double h, V0, k1, k2, k3;
    float *out;
};
hipError_t launch_bold(const BoldArgs &a, hipStream_t s);

// Optional per-kernel timing of the analysis launches (HIP events on the
// launch stream): transpose, Welch, analytic signal, PLI, Up/Down, final.
constexpr int kAnKernels = 6;
struct AnTimer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[kAnKernels];
    int64_t n[kAnKernels] = {};
    double ms[kAnKernels] = {};
};

// Host driver shared by the two entry points: instances given by their
// sample offsets (floats from `samples`) and region counts.
struct AnInstances {
    const float *samples;
    const int64_t *samp_off;
    const int32_t *n;
    int64_t n_inst;
    int64_t n_samples;
};
vadx_status run_analysis(int device, hipStream_t stream, const AnInstances &in, double period_ms,
                         const vadx_analysis_cfg *cfg, void *ws, size_t ws_bytes,
                         vadx_analysis *out, float *psd_out, float *pli_out, AnTimer *timer,
                         std::string &err);
vadx_status analysis_bytes(int64_t n_samples, int32_t n_max, int64_t regions_per_pass,
                           const vadx_analysis_cfg *cfg, size_t *bytes, std::string &err);

} // namespace vadx
