// bold.hip -- Balloon-Windkessel BOLD signal of every region from its stored
// excitatory rate samples (Section 2.4; haemodynamics after Stephan et al.
// 2007 with the classical output coefficients). One thread per region walks
// the samples in the stored [t][n] layout (the lanes of one instance read
// consecutive addresses): classical Runge-Kutta with the sample period as the
// step, the rate (kHz) held over each sample as the neural input, the state in
// double precision and its derivatives in single precision.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "analysis_engine.h"

namespace vadx {

namespace {

struct BoldRhs {
    float kappa, gamma, inv_tau0, inv_alpha, inv_E0, l2_1mE0;   // l2_1mE0 = log2(1 - E0)
};

__device__ inline void bold_rhs(const BoldRhs &p, float z, float s, float f, float v, float q,
                                float d[4])
{
    const float vpow = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(v) * p.inv_alpha);   // v^(1/alpha)
    const float ext = 1.f - __builtin_amdgcn_exp2f(p.l2_1mE0 * __builtin_amdgcn_rcpf(f)); // 1 - (1-E0)^(1/f)
    d[0] = z - p.kappa * s - p.gamma * (f - 1.f);
    d[1] = s;
    d[2] = (f - vpow) * p.inv_tau0;
    d[3] = (f * ext * p.inv_E0 - vpow * q * __builtin_amdgcn_rcpf(v)) * p.inv_tau0;
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
    p.inv_alpha = a.inv_alpha;
    p.inv_E0 = a.inv_E0;
    p.l2_1mE0 = a.l2_1mE0;
    const double h = a.h, h2 = 0.5 * a.h, h6 = a.h / 6.0;
    double X[4] = {0.0, 1.0, 1.0, 1.0};
    int m = 0;
    int next = a.n_tr > 0 ? a.emit[0] : -1;
    for (int64_t t = 0; t < a.n_samples; ++t) {
        const float z = x[t * n];
        float k1[4], k2[4], k3[4], k4[4];
        double Y[4];
        bold_rhs(p, z, (float)X[0], (float)X[1], (float)X[2], (float)X[3], k1);
#pragma unroll
        for (int c = 0; c < 4; ++c) Y[c] = X[c] + h2 * (double)k1[c];
        bold_rhs(p, z, (float)Y[0], (float)Y[1], (float)Y[2], (float)Y[3], k2);
#pragma unroll
        for (int c = 0; c < 4; ++c) Y[c] = X[c] + h2 * (double)k2[c];
        bold_rhs(p, z, (float)Y[0], (float)Y[1], (float)Y[2], (float)Y[3], k3);
#pragma unroll
        for (int c = 0; c < 4; ++c) Y[c] = X[c] + h * (double)k3[c];
        bold_rhs(p, z, (float)Y[0], (float)Y[1], (float)Y[2], (float)Y[3], k4);
#pragma unroll
        for (int c = 0; c < 4; ++c)
            X[c] += h6 * ((double)k1[c] + 2.0 * (double)k2[c] + 2.0 * (double)k3[c] + (double)k4[c]);
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
