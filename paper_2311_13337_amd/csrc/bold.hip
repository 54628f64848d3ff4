// bold.hip -- Balloon-Windkessel BOLD signal of every region from its stored
// excitatory rate samples (Section 2.4; haemodynamics after Stephan et al.
// 2007 with the classical output coefficients). One thread per region walks
// the samples in the stored [t][n] layout (the lanes of one instance read
// consecutive addresses): classical Runge-Kutta with the sample period as the
// step, the rate (kHz) held over each sample as the neural input, the state and
// its update in double precision, the stage states and derivatives in single.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "analysis_engine.h"

namespace vadx {

namespace {

struct BoldRhs {
    float kappa, gamma, inv_tau0, inv_alpha_m1, E0tau, l2_1mE0;   // 1/alpha - 1, 1/(E0 tau0), log2(1 - E0)
};

// The four derivatives of (s, f, v, q) with the neural input z. v^(1/alpha)
// is taken as v * v^(1/alpha - 1), so that vpow q / v needs no reciprocal.
__device__ inline void bold_rhs(const BoldRhs &p, float z, float s, float f, float v, float q,
                                float d[4])
{
    const float vpow_v = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(v) * p.inv_alpha_m1);   // v^(1/alpha - 1)
    const float vpow = vpow_v * v;
    const float ext = 1.f - __builtin_amdgcn_exp2f(p.l2_1mE0 * __builtin_amdgcn_rcpf(f));     // 1 - (1-E0)^(1/f)
    d[0] = z - p.kappa * s - p.gamma * (f - 1.f);
    d[1] = s;
    d[2] = (f - vpow) * p.inv_tau0;
    d[3] = f * ext * p.E0tau - vpow_v * q * p.inv_tau0;
}

} // namespace

__global__ __launch_bounds__(256) void bold_kernel(BoldArgs a)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= a.n_reg) return;
    const int i = a.reg_inst[g];
    const int n = a.n[i];
    const int k = (int)(g - a.rbase[i]);
    const float *x = a.samples + a.samp_off[i] + k;
    float *out = a.out + a.out_off[i] + k;
    BoldRhs p;
    p.kappa = a.kappa;
    p.gamma = a.gamma;
    p.inv_tau0 = a.inv_tau0;
    p.inv_alpha_m1 = a.inv_alpha - 1.f;
    p.E0tau = a.inv_E0 * a.inv_tau0;
    p.l2_1mE0 = a.l2_1mE0;
    const float hf = (float)a.h, h2f = 0.5f * hf;
    const double h6 = a.h / 6.0;
    // The state in double; each step's stage states are formed in single
    // precision from the state rounded once, as the derivatives take them.
    double X[4] = {0.0, 1.0, 1.0, 1.0};
    int m = 0;
    int next = a.n_tr > 0 ? a.emit[0] : -1;
    // each sample is loaded one step before it is used (the last load repeats
    // the last sample, staying in bounds)
    float znext = a.n_samples > 0 ? *x : 0.f;
    for (int64_t t = 0; t < a.n_samples; ++t) {
        const float z = znext;
        x += t + 1 < a.n_samples ? n : 0;
        znext = *x;
        float Xf[4], k1[4], k2[4], k3[4], k4[4], Y[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) Xf[c] = (float)X[c];
        bold_rhs(p, z, Xf[0], Xf[1], Xf[2], Xf[3], k1);
#pragma unroll
        for (int c = 0; c < 4; ++c) Y[c] = Xf[c] + h2f * k1[c];
        bold_rhs(p, z, Y[0], Y[1], Y[2], Y[3], k2);
#pragma unroll
        for (int c = 0; c < 4; ++c) Y[c] = Xf[c] + h2f * k2[c];
        bold_rhs(p, z, Y[0], Y[1], Y[2], Y[3], k3);
#pragma unroll
        for (int c = 0; c < 4; ++c) Y[c] = Xf[c] + hf * k3[c];
        bold_rhs(p, z, Y[0], Y[1], Y[2], Y[3], k4);
#pragma unroll
        for (int c = 0; c < 4; ++c) X[c] += h6 * (double)((k1[c] + k4[c]) + 2.f * (k2[c] + k3[c]));
        while (next >= 0 && t + 1 >= next) {
            const double y = a.V0 * (a.k1 * (1.0 - X[3]) + a.k2 * (1.0 - X[3] / X[2]) +
                                     a.k3 * (1.0 - X[2]));
            out[(int64_t)m * n] = (float)y;
            ++m;
            next = m < a.n_tr ? a.emit[m] : -1;
        }
    }
}

hipError_t launch_bold(const BoldArgs &a, hipStream_t s)
{
    if (a.n_reg == 0) return hipSuccess;
    hipLaunchKernelGGL(bold_kernel, dim3((unsigned)((a.n_reg + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

} // namespace vadx
