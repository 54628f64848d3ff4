// Host build of the GPU model arithmetic (adex_model.h instantiated with float
// and double state, as in the integration kernel) for checks against the FP64
// oracle on machines without a GPU. Test infrastructure only.
#include "adex_model.h"
#include "kmodel.h"
#include "vadx.h"

using namespace vadx;

extern "C" {

// Value, gradient, Hessian (from q with C = 2 e_e e_e^T, 2 e_i e_i^T and
// e_e e_i^T + e_i e_e^T) and mu_V of one population's transfer function.
void mh_tf(const vadx_model *m, int pop, float xe, float xi, float W, float *out)
{
    KModel k = make_kmodel(*m);
    float mu = 0.f;
    const float cs[3][3] = {{2.f, 0.f, 0.f}, {0.f, 1.f, 0.f}, {0.f, 0.f, 2.f}};
    float hq[3];
    QJet<float> F{};
    for (int t = 0; t < 3; ++t) {
        Cov<float> C;
        C.ee = cs[t][0];
        C.ei = cs[t][1];
        C.ii = cs[t][2];
        cvec(C, k.aE, k.aI, C.nx, C.ny);
        C.qG = 0.5f * (k.aE * C.nx + k.aI * C.ny);
        if (m->tau_e == m->tau_i)
            F = transfer<true>(k, pop, tf_shared<true>(k, xe, xi, C), C, W, mu);
        else
            F = transfer<false>(k, pop, tf_shared<false>(k, xe, xi, C), C, W, mu);
        hq[t] = F.q;
    }
    out[0] = F.v; out[1] = F.a; out[2] = F.b; out[3] = hq[0]; out[4] = hq[1]; out[5] = hq[2];
    out[6] = mu;
}

void mh_drift(const vadx_model *m, const float *X, float c, float be, float ae, float *dX)
{
    KModel k = make_kmodel(*m);
    switch (model_variant(k)) {
    case 0: drift<0>(k, X, c, inst_model(k, be, ae), dX); break;
    case 1: drift<1>(k, X, c, inst_model(k, be, ae), dX); break;
    case 2: drift<2>(k, X, c, inst_model(k, be, ae), dX); break;
    default: drift<3>(k, X, c, inst_model(k, be, ae), dX); break;
    }
}

int mh_step(const vadx_model *m, int integrator, double dt, double *X, float c, float be, float ae,
            double gdw)
{
    KModel k = make_kmodel(*m);
    switch (model_variant(k)) {
    case 0: return step_region<0>(k, integrator, dt, X, c, inst_model(k, be, ae), gdw);
    case 1: return step_region<1>(k, integrator, dt, X, c, inst_model(k, be, ae), gdw);
    case 2: return step_region<2>(k, integrator, dt, X, c, inst_model(k, be, ae), gdw);
    default: return step_region<3>(k, integrator, dt, X, c, inst_model(k, be, ae), gdw);
    }
}

} // extern "C"
