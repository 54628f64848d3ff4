// mlp_engine.h -- device layout and launchers of the surrogate network
// (internal to libvadx).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "vadx.h"

namespace vadx {

constexpr int kMlpTile = 32;            // samples per workgroup
constexpr int kMlpParams = 17926;       // W1 128x4, b1 128, W2 128x128, b2 128, W3 6x128, b3 6
constexpr int kMlpOffW1 = 0, kMlpOffB1 = 512, kMlpOffW2 = 640, kMlpOffB2 = 17024;
constexpr int kMlpOffW3 = 17152, kMlpOffB3 = 17920, kMlpOffLoss = 17926;
constexpr int kMlpSlot = 17984;         // per-tile gradient slot (params + loss, padded)

struct MlpArgs {
    float *params, *m, *v, *grad, *partial, *loss_out;
    float x_lo[4], x_scale[4];          // x_n = (x - lo) * scale - 1, scale = 2 / (hi - lo)
    float y_mean[6], y_rstd[6], y_std[6];
    float lr, beta1, beta2, eps;
    int score_out0, score_out1;         // outputs whose input gradients form the score
};

hipError_t launch_mlp_grad(const MlpArgs &a, const float *X, const float *Y, int n, int n_total,
                           hipStream_t s);
hipError_t launch_mlp_adam(const MlpArgs &a, int n_tiles, float c1, float c2, int apply, int step,
                           hipStream_t s);
hipError_t launch_mlp_predict(const MlpArgs &a, const float *X, int64_t n, float *Y, float *J,
                              float *score, hipStream_t s);

// screening selection (select.hip)
int64_t select_tiles(int64_t n);
hipError_t launch_sel_hist(const float *score, int64_t n, uint32_t prefix, uint32_t mask, int shift,
                           uint32_t *hist, hipStream_t s);
hipError_t launch_sel_compact(const float *score, int64_t n, int phase, int use_top, uint32_t T,
                              int64_t need, float audit_frac, uint32_t seed, const int64_t *eq_base,
                              const int64_t *sel_base, uint32_t *out, int64_t *sel,
                              uint8_t *is_audit, hipStream_t s);

// Device scratch of the selection (grown on demand, owned by the caller).
struct SelScratch {
    void *p = nullptr;
    int64_t tiles = -1;
};
// The k largest scores (ties to the lower index) plus an audit sample of the
// rest (probability audit_frac, Philox keyed (seed, index)), indices ascending;
// synchronises s.
// With host_counts / host_bases (select_tiles(n) entries each, nullable) the
// per-tile host staging uses them instead of allocating; a scratch `sc` of at
// least select_tiles(n) tiles is used as it is (no device allocation).
vadx_status select_run(hipStream_t s, SelScratch &sc, const float *score, int64_t n, int64_t k,
                       float audit_frac, uint32_t seed, int64_t *sel, uint8_t *is_audit,
                       int64_t capacity, int64_t *n_sel, std::string &err,
                       uint32_t *host_counts = nullptr, int64_t *host_bases = nullptr);
// Bytes of a selection scratch of `tiles` tiles (layout of select_run).
size_t select_scratch_bytes(int64_t tiles);

} // namespace vadx
