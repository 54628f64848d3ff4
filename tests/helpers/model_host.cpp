// Host build of the GPU model arithmetic (adex_model.h instantiated with float
// and double state, as in the integration kernel) for checks against the FP64
// oracle on machines without a GPU. Test infrastructure only.
#include "adex_model.h"
#include "kmodel.h"
#include "vadx.h"

using namespace vadx;

extern "C" {

void mh_tf(const vadx_model *m, int pop, float xe, float xi, float W, float *out)
{
    KModel k = make_kmodel(*m);
    float mu = 0.f;
    Jet<float> F;
    if (m->tau_e == m->tau_i)
        F = transfer<true>(k, pop, tf_shared<true>(k, xe, xi), W, mu);
    else
        F = transfer<false>(k, pop, tf_shared<false>(k, xe, xi), W, mu);
    out[0] = F.v; out[1] = F.a; out[2] = F.b; out[3] = F.aa; out[4] = F.ab; out[5] = F.bb; out[6] = mu;
}

void mh_drift(const vadx_model *m, const float *X, float c, float be, float ae, float *dX)
{
    KModel k = make_kmodel(*m);
    switch (model_variant(k)) {
    case 0: drift<0>(k, X, c, be, ae, dX); break;
    case 1: drift<1>(k, X, c, be, ae, dX); break;
    case 2: drift<2>(k, X, c, be, ae, dX); break;
    default: drift<3>(k, X, c, be, ae, dX); break;
    }
}

int mh_step(const vadx_model *m, int integrator, double dt, double *X, float c, float be, float ae,
            double gdw)
{
    KModel k = make_kmodel(*m);
    switch (model_variant(k)) {
    case 0: return step_region<0>(k, integrator, dt, X, c, be, ae, gdw);
    case 1: return step_region<1>(k, integrator, dt, X, c, be, ae, gdw);
    case 2: return step_region<2>(k, integrator, dt, X, c, be, ae, gdw);
    default: return step_region<3>(k, integrator, dt, X, c, be, ae, gdw);
    }
}

} // extern "C"
