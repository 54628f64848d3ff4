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
    Jet<float> F = m->tau_e == m->tau_i ? transfer<true>(k, pop, xe, xi, W, mu)
                                        : transfer<false>(k, pop, xe, xi, W, mu);
    out[0] = F.v; out[1] = F.a; out[2] = F.b; out[3] = F.aa; out[4] = F.ab; out[5] = F.bb; out[6] = mu;
}

void mh_drift(const vadx_model *m, const float *X, float c, float be, float ae, float *dX)
{
    KModel k = make_kmodel(*m);
    if (m->tau_e == m->tau_i) drift<true>(k, X, c, be, ae, dX);
    else drift<false>(k, X, c, be, ae, dX);
}

int mh_step(const vadx_model *m, int integrator, double dt, double *X, float c, float be, float ae,
            double gdw)
{
    KModel k = make_kmodel(*m);
    return m->tau_e == m->tau_i ? step_region<true>(k, integrator, dt, X, c, be, ae, gdw)
                                : step_region<false>(k, integrator, dt, X, c, be, ae, gdw);
}

} // extern "C"
