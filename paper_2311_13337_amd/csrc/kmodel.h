// kmodel.h -- host-side derivation of the FP32 model constants (KModel) from
// the double-precision vadx_model: unit products and the threshold polynomial
// of Table 1 re-expressed in raw (mu_V, sqrt2 sigma_V, tau_V) offsets from the
// centre of its normalisation.
#pragma once
#include <cmath>

#include "adex_model.h"
#include "vadx.h"

namespace vadx {

inline KModel make_kmodel(const vadx_model &m)
{
    KModel k{};
    k.aE = (float)(m.Q_e * m.tau_e * m.K_e);
    k.aI = (float)(m.Q_i * m.tau_i * m.K_i);
    k.gL = (float)m.g_L; k.Cm = (float)m.C_m; k.Ee = (float)m.E_e; k.Ei = (float)m.E_i;
    k.tau_e = (float)m.tau_e; k.tau_i = (float)m.tau_i;
    k.ce = (float)(m.K_e * m.tau_e * m.tau_e * m.Q_e * m.Q_e);
    k.ci = (float)(m.K_i * m.tau_i * m.tau_i * m.Q_i * m.Q_i);
    {
        const double aE = m.Q_e * m.tau_e * m.K_e, aI = m.Q_i * m.tau_i * m.K_i;
        const double ce = m.K_e * m.tau_e * m.tau_e * m.Q_e * m.Q_e;
        const double ci = m.K_i * m.tau_i * m.tau_i * m.Q_i * m.Q_i;
        const double bE = aI * (m.E_e - m.E_i), bI = aE * (m.E_i - m.E_e);
        k.aEE = (float)(aE * aE); k.aEI = (float)(aE * aI); k.aII = (float)(aI * aI);
        k.bE = (float)bE; k.bI = (float)bI;
        k.EegL = (float)(m.E_e * m.g_L); k.EigL = (float)(m.E_i * m.g_L);
        k.ce2bE = (float)(2 * ce * bE); k.ci2bI = (float)(2 * ci * bI);
        k.ce2bE2 = (float)(2 * ce * bE * bE); k.ci2bI2 = (float)(2 * ci * bI * bI);
    }
    k.EL[0] = (float)m.E_L_e; k.EL[1] = (float)m.E_L_i;
    k.gLEL[0] = (float)(m.g_L * m.E_L_e); k.gLEL[1] = (float)(m.g_L * m.E_L_i);
    // Table 1 evaluates the polynomial in normalised coordinates
    // n = ((mu_V - muV0)/dmuV0, (sigma_V - sV0)/dsV0, (tau_N - tN0)/dtN0) with
    // tau_N = tau_V g_L / C_m; in u = (mu_V, sqrt2 sigma_V, tau_V) that is
    // n_k = s_k (u_k - c_k)
    const double sc[3] = {1.0 / m.dmuV0, 1.0 / (std::sqrt(2.0) * m.dsV0), m.g_L / (m.C_m * m.dtN0)};
    const double cc[3] = {m.muV0, std::sqrt(2.0) * m.sV0, m.tN0 * m.C_m / m.g_L};
    for (int i = 0; i < 3; ++i) k.pc[i] = (float)cc[i];
    for (int p = 0; p < 2; ++p) {
        const double *P = p == 0 ? m.P_e : m.P_i;
        // Table 1 order: P0, P_mu, P_sigma, P_tau, P_mu^2, P_sigma^2, P_tau^2,
        // P_mu sigma, P_mu tau, P_sigma tau (the last three are cross terms)
        const double H[3][3] = {{2 * P[4], P[7], P[8]}, {P[7], 2 * P[5], P[9]}, {P[8], P[9], 2 * P[6]}};
        k.P0[p] = (float)P[0];
        for (int i = 0; i < 3; ++i) k.plin[p][i] = (float)(P[1 + i] * sc[i]);
        int q = 0;
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j) {
                k.Hraw[p][q] = (float)(sc[i] * sc[j] * H[i][j]);
                k.Hq[p][q] = (float)((i == j ? 0.5 : 1.0) * sc[i] * sc[j] * H[i][j]);
                ++q;
            }
    }
    k.invT = (float)(1.0 / m.T); k.invNe = (float)(1.0 / m.N_e); k.invNi = (float)(1.0 / m.N_i);
    k.inv_tauw[0] = (float)(1.0 / m.tau_w_e); k.inv_tauw[1] = (float)(1.0 / m.tau_w_i);
    k.b_i = (float)m.b_i; k.a_i = (float)m.a_i;
    k.cF[0][0] = (float)m.cF_ee; k.cF[0][1] = (float)m.cF_ei;
    k.cF[1][0] = (float)m.cF_ie; k.cF[1][1] = (float)m.cF_ii;
    k.same_inputs = k.cF[0][0] == k.cF[1][0] && k.cF[0][1] == k.cF[1][1];
    k.inv_tauOU = (float)(1.0 / m.tau_OU);
    k.w_noise = (float)m.w_noise; k.rate_max = (float)m.rate_max; k.x_floor = (float)m.x_floor;
    return k;
}

} // namespace vadx
