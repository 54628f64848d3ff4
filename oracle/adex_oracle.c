/*
 * adex_oracle.c -- plain, slow FP64 CPU oracle of the TVB-AdEx sweep hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it. It shares no code, header, table or constant with the GPU
 * library.
 *
 * What it computes (van der Vlag et al., "Vast TVB parameter space
 * exploration", arXiv:2311.13337):
 *   - the second-order AdEx mean field, eq. (1)-(3) of Section 2.1, with the
 *     derivatives of the transfer function taken exactly by second-order
 *     forward-mode jets (hyper-dual numbers) in the two excitatory/inhibitory
 *     input rates;
 *   - the transfer function of Section 2.2: the semi-analytic template in
 *     (mu_V, sigma_V, tau_V), the phenomenological threshold polynomial of
 *     Table 1 and the normal-law firing estimate; its inputs are eq. (5):
 *     delayed, weighted excitatory rates of the other regions, OU noise and
 *     constant drives;
 *   - Ornstein-Uhlenbeck noise, eq. (4), driven by Philox4x32-10 normals;
 *   - delayed linear coupling with delays = tract length / speed (Section 2.2);
 *   - stochastic Heun time stepping, time-averaged rate samples (Section 2.4)
 *     and the Pearson functional connectivity, eq. (6), with the summary
 *     statistics built on it.
 * Readings of points the paper leaves open are the ones listed in the design
 * notes of this repository (integrator, units in kHz, initial state, clamps,
 * noise realisation, statistics definitions).
 *
 * No blocking, no fusion, no ring buffer: the full rate history is kept.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Model constants (one struct; field order mirrored by the Python shim).     */
/* ------------------------------------------------------------------------- */
typedef struct {
    double C_m, g_L, E_e, E_i, Q_e, Q_i, tau_e, tau_i, K_e, K_i, N_e, N_i, T;
    double E_L_e, E_L_i, tau_w_e, tau_w_i, b_i, a_i;
    double cF_ee, cF_ei, cF_ie, cF_ii;
    double tau_OU, sigma_OU, w_noise;
    double muV0, dmuV0, sV0, dsV0, tN0, dtN0;
    double rate_max, E_init, I_init, x_floor;
    double P_e[10], P_i[10];
    /* Transfer-function kind: 0 = the semi-analytic template (the model);
       1 = a quadratic test function F = F0 + g.x + x^T H x / 2, used only
       to pin the moment equations (1)-(2) against closed forms. */
    int64_t tf_kind;
    double q_F0[2], q_g[2][2], q_H[2][3]; /* per population: H_ee, H_ei, H_ii */
} or_model;

enum { ORACLE_PRESET_LITERATURE_B = 0, ORACLE_PRESET_PAPER_T1 = 1 };

/* Threshold polynomial coefficients, Table 1 (mV), column order
   P0, P_muV, P_sigmaV, P_tauNV, P_mu2, P_sigma2, P_tauNV2, P_Vsigma, P_muVtauN,
   P_sigmaVtauN. */
static const double T1_RS[10] = {-48.9, 5.1, -25.0, 1.4, -0.41, 10.5, -36.0, 7.4, 1.2, 40.7};
static const double T1_FS[10] = {-51.4, 0.4, -8.3, 0.2, -0.5, 1.4, -14.6, 4.5, 2.8, 15.3};

int oracle_model_preset(int preset, or_model *m)
{
    if (preset != ORACLE_PRESET_LITERATURE_B && preset != ORACLE_PRESET_PAPER_T1) return -1;
    memset(m, 0, sizeof(*m));
    m->C_m = 200.0;   m->g_L = 10.0;   m->E_e = 0.0;   m->E_i = -80.0;
    m->Q_e = 1.5;     m->Q_i = 5.0;    m->tau_e = 5.0; m->tau_i = 5.0;
    /* K = p_connect * N_tot * (1-g) resp. g with p=0.05, N_tot=1e4, g=0.2 */
    m->K_e = 400.0;   m->K_i = 100.0;  m->N_e = 8000.0; m->N_i = 2000.0;
    m->T = 20.0;
    m->E_L_e = -64.0; m->E_L_i = -65.0;
    m->tau_w_e = 500.0; m->tau_w_i = 1.0; m->b_i = 0.0; m->a_i = 0.0;
    /* external drives (kHz): the upper end of Table 4's range for the
       excitatory inputs. With the lower end (0.3e-3) the node keeps a
       quiescent fixed point near 4e-8 Hz that absorbs most networks with
       b_e >= 48 pA, so the sweep box has no synchronous regime; at 0.5e-3
       that state is gone and adaptation turns the active state into slow
       oscillations (Section 3.2.1). */
    m->cF_ee = 0.5e-3; m->cF_ei = 0.0; m->cF_ie = 0.5e-3; m->cF_ii = 0.0;
    m->tau_OU = 5.0;  m->sigma_OU = 1e-3; m->w_noise = 1e-3;
    m->muV0 = -60.0;  m->dmuV0 = 10.0; m->sV0 = 4.0; m->dsV0 = 6.0;
    m->tN0 = 0.5;     m->dtN0 = 1.0;
    m->rate_max = 1.0; m->E_init = 0.004; m->I_init = 0.01;
    /* minimum input rate of the transfer function (kHz): spontaneous release */
    m->x_floor = 1e-6;
    memcpy(m->P_e, T1_RS, sizeof(T1_RS));
    memcpy(m->P_i, T1_FS, sizeof(T1_FS));
    if (preset == ORACLE_PRESET_LITERATURE_B) {
        /* Reading of Table 1 as garbled in three places: RS P0 digits swapped,
           FS P_muV off by a decade, and the sigma*tau cross-terms of both
           cells with the wrong sign. */
        m->P_e[0] = -49.8;
        m->P_i[1] = 4.0;
        m->P_e[9] = -m->P_e[9];
        m->P_i[9] = -m->P_i[9];
    }
    m->tf_kind = 0;
    return 0;
}

size_t oracle_model_size(void) { return sizeof(or_model); }

/* ------------------------------------------------------------------------- */
/* Second-order jets in the two input rates (x_e, x_i).                       */
/* v = value, a = d/dx_e, b = d/dx_i, aa, ab, bb = second derivatives.        */
/* ------------------------------------------------------------------------- */
typedef struct { double v, a, b, aa, ab, bb; } jet;

static jet j_const(double c) { jet r = {c, 0, 0, 0, 0, 0}; return r; }
static jet j_var_a(double x) { jet r = {x, 1, 0, 0, 0, 0}; return r; }
static jet j_var_b(double x) { jet r = {x, 0, 1, 0, 0, 0}; return r; }

static jet j_add(jet x, jet y)
{
    jet r = {x.v + y.v, x.a + y.a, x.b + y.b, x.aa + y.aa, x.ab + y.ab, x.bb + y.bb};
    return r;
}
static jet j_sub(jet x, jet y)
{
    jet r = {x.v - y.v, x.a - y.a, x.b - y.b, x.aa - y.aa, x.ab - y.ab, x.bb - y.bb};
    return r;
}
static jet j_scale(jet x, double s)
{
    jet r = {s * x.v, s * x.a, s * x.b, s * x.aa, s * x.ab, s * x.bb};
    return r;
}
static jet j_addc(jet x, double c) { x.v += c; return x; }

/* Product rule to second order. */
static jet j_mul(jet x, jet y)
{
    jet r;
    r.v = x.v * y.v;
    r.a = x.a * y.v + x.v * y.a;
    r.b = x.b * y.v + x.v * y.b;
    r.aa = x.aa * y.v + 2.0 * x.a * y.a + x.v * y.aa;
    r.ab = x.ab * y.v + x.a * y.b + x.b * y.a + x.v * y.ab;
    r.bb = x.bb * y.v + 2.0 * x.b * y.b + x.v * y.bb;
    return r;
}

/* Chain rule for a scalar function f with f(x.v)=f0, f'=f1, f''=f2. */
static jet j_chain(jet x, double f0, double f1, double f2)
{
    jet r;
    r.v = f0;
    r.a = f1 * x.a;
    r.b = f1 * x.b;
    r.aa = f1 * x.aa + f2 * x.a * x.a;
    r.ab = f1 * x.ab + f2 * x.a * x.b;
    r.bb = f1 * x.bb + f2 * x.b * x.b;
    return r;
}

static jet j_recip(jet x)
{
    double u = 1.0 / x.v;
    return j_chain(x, u, -u * u, 2.0 * u * u * u);
}
static jet j_div(jet x, jet y) { return j_mul(x, j_recip(y)); }
static jet j_sqrt(jet x)
{
    double s = sqrt(x.v);
    return j_chain(x, s, 0.5 / s, -0.25 / (s * x.v));
}
static jet j_erfc(jet x)
{
    const double two_over_sqrtpi = 1.1283791670955126;
    double g1 = -two_over_sqrtpi * exp(-x.v * x.v);
    return j_chain(x, erfc(x.v), g1, -2.0 * x.v * g1);
}

/* ------------------------------------------------------------------------- */
/* Transfer function (Section 2.2).                                           */
/* ------------------------------------------------------------------------- */
typedef struct { jet F; double muV, sigV, tauV, Vthre; } tf_out;

/* pop 0 = excitatory (RS cell, E_L_e, W_e), 1 = inhibitory (FS cell, E_L_i, W_i).
   xe, xi: total excitatory / inhibitory input rates (kHz), already floored.
   W: adaptation current (pA). Derivatives are taken in (xe, xi). */
static tf_out tf_eval(const or_model *m, int pop, double xe, double xi, double W)
{
    tf_out o;
    memset(&o, 0, sizeof(o));
    if (m->tf_kind == 1) {
        jet X = j_var_a(xe), Y = j_var_b(xi);
        const double *g = m->q_g[pop], *H = m->q_H[pop];
        jet F = j_const(m->q_F0[pop]);
        F = j_add(F, j_add(j_scale(X, g[0]), j_scale(Y, g[1])));
        F = j_add(F, j_scale(j_mul(X, X), 0.5 * H[0]));
        F = j_add(F, j_scale(j_mul(X, Y), H[1]));
        F = j_add(F, j_scale(j_mul(Y, Y), 0.5 * H[2]));
        o.F = F;
        return o;
    }
    const double E_L = pop == 0 ? m->E_L_e : m->E_L_i;
    const double *P = pop == 0 ? m->P_e : m->P_i;

    jet Xe = j_var_a(xe), Xi = j_var_b(xi);
    /* mean conductances (nS), total conductance, effective time constant */
    jet muGe = j_scale(Xe, m->Q_e * m->tau_e * m->K_e);
    jet muGi = j_scale(Xi, m->Q_i * m->tau_i * m->K_i);
    jet muG = j_addc(j_add(muGe, muGi), m->g_L);
    jet Teff = j_div(j_const(m->C_m), muG);
    /* mean membrane potential (mV): conductance-weighted reversal potentials */
    jet num = j_addc(j_add(j_scale(muGe, m->E_e), j_scale(muGi, m->E_i)), m->g_L * E_L - W);
    jet muV = j_div(num, muG);
    /* PSP amplitudes (mV) */
    jet Ue = j_div(j_scale(j_sub(j_const(m->E_e), muV), m->Q_e), muG);
    jet Ui = j_div(j_scale(j_sub(j_const(m->E_i), muV), m->Q_i), muG);
    /* shot-noise weights: rate x (U tau)^2 */
    jet Uet = j_scale(Ue, m->tau_e), Uit = j_scale(Ui, m->tau_i);
    jet Ae = j_mul(j_scale(Xe, m->K_e), j_mul(Uet, Uet));
    jet Ai = j_mul(j_scale(Xi, m->K_i), j_mul(Uit, Uit));
    o.muV = muV.v;
    if (xe == 0.0 && xi == 0.0) {
        /* no input: no fluctuations, no firing; F and its derivatives are 0 */
        o.F = j_const(0.0);
        return o;
    }
    jet de = j_recip(j_addc(Teff, m->tau_e));
    jet di = j_recip(j_addc(Teff, m->tau_i));
    jet Ade = j_mul(Ae, de), Adi = j_mul(Ai, di);
    jet sV = j_sqrt(j_scale(j_add(Ade, Adi), 0.5));
    jet TV = j_div(j_add(Ae, Ai), j_add(Ade, Adi));
    jet TN = j_scale(TV, m->g_L / m->C_m);
    /* normalised coordinates of the threshold polynomial */
    jet mm = j_scale(j_addc(muV, -m->muV0), 1.0 / m->dmuV0);
    jet ss = j_scale(j_addc(sV, -m->sV0), 1.0 / m->dsV0);
    jet tt = j_scale(j_addc(TN, -m->tN0), 1.0 / m->dtN0);
    jet V = j_const(P[0]);
    V = j_add(V, j_scale(mm, P[1]));
    V = j_add(V, j_scale(ss, P[2]));
    V = j_add(V, j_scale(tt, P[3]));
    V = j_add(V, j_scale(j_mul(mm, mm), P[4]));
    V = j_add(V, j_scale(j_mul(ss, ss), P[5]));
    V = j_add(V, j_scale(j_mul(tt, tt), P[6]));
    V = j_add(V, j_scale(j_mul(mm, ss), P[7]));
    V = j_add(V, j_scale(j_mul(mm, tt), P[8]));
    V = j_add(V, j_scale(j_mul(ss, tt), P[9]));
    /* normal-law estimate: F = erfc((V_thre - muV) / (sqrt2 sigma_V)) / (2 tau_V) */
    jet z = j_div(j_sub(V, muV), j_scale(sV, sqrt(2.0)));
    o.F = j_div(j_erfc(z), j_scale(TV, 2.0));
    o.sigV = sV.v;
    o.tauV = TV.v;
    o.Vthre = V.v;
    return o;
}

/* Python entry: out[0..5] = F jet (v, d/dxe, d/dxi, d2/dxe2, d2/dxedxi, d2/dxi2),
   out[6..9] = muV, sigmaV, tauV, Vthre. */
void oracle_tf(const or_model *m, int pop, double xe, double xi, double W, double *out)
{
    tf_out o = tf_eval(m, pop, xe, xi, W);
    out[0] = o.F.v;  out[1] = o.F.a;  out[2] = o.F.b;
    out[3] = o.F.aa; out[4] = o.F.ab; out[5] = o.F.bb;
    out[6] = o.muV;  out[7] = o.sigV; out[8] = o.tauV; out[9] = o.Vthre;
}

/* ------------------------------------------------------------------------- */
/* Drift of one region (eq. 1-4).                                             */
/* State order: E, I, C_ee, C_ei, C_ii, W_e, W_i, OU (rates in kHz).          */
/* ------------------------------------------------------------------------- */
enum { SV_E = 0, SV_I, SV_CEE, SV_CEI, SV_CII, SV_WE, SV_WI, SV_OU, N_SV };

void oracle_drift(const or_model *m, const double *X, double c, double b_e, double a_e,
                  double *dX)
{
    const double E = X[SV_E], I = X[SV_I];
    const double noise = m->w_noise * X[SV_OU];
    /* TF inputs per population, eq. (5): delayed coupling + noise + drive on
       the excitatory input, local inhibitory rate + drive on the inhibitory one */
    double xe[2], xi[2], Wp[2];
    xe[0] = fmax(E + c + noise + m->cF_ee, m->x_floor);
    xi[0] = fmax(I + m->cF_ei, m->x_floor);
    xe[1] = fmax(E + c + noise + m->cF_ie, m->x_floor);
    xi[1] = fmax(I + m->cF_ii, m->x_floor);
    Wp[0] = X[SV_WE];
    Wp[1] = X[SV_WI];
    tf_out tf[2];
    for (int p = 0; p < 2; ++p) tf[p] = tf_eval(m, p, xe[p], xi[p], Wp[p]);

    /* index form of eq. (1)-(2): lambda, eta, mu in {e, i} */
    double nu[2] = {E, I};
    double Nn[2] = {m->N_e, m->N_i};
    double C[2][2] = {{X[SV_CEE], X[SV_CEI]}, {X[SV_CEI], X[SV_CII]}};
    double F[2], J[2][2], H[2][2][2];
    for (int p = 0; p < 2; ++p) {
        F[p] = tf[p].F.v;
        J[p][0] = tf[p].F.a;
        J[p][1] = tf[p].F.b;
        H[p][0][0] = tf[p].F.aa;
        H[p][0][1] = tf[p].F.ab;
        H[p][1][0] = tf[p].F.ab;
        H[p][1][1] = tf[p].F.bb;
    }
    const double T = m->T;
    double dnu[2];
    for (int mu = 0; mu < 2; ++mu) {
        double s = 0.0;
        for (int l = 0; l < 2; ++l)
            for (int h = 0; h < 2; ++h) s += C[l][h] * H[mu][l][h];
        dnu[mu] = ((F[mu] - nu[mu]) + 0.5 * s) / T;
    }
    double dC[2][2];
    for (int l = 0; l < 2; ++l)
        for (int h = 0; h < 2; ++h) {
            double r = (l == h) ? F[l] * (1.0 / T - F[h]) / Nn[l] : 0.0;
            r += (F[l] - nu[l]) * (F[h] - nu[h]);
            for (int mu = 0; mu < 2; ++mu) r += J[l][mu] * C[h][mu] + J[h][mu] * C[l][mu];
            r -= 2.0 * C[l][h];
            dC[l][h] = r / T;
        }
    dX[SV_E] = dnu[0];
    dX[SV_I] = dnu[1];
    dX[SV_CEE] = dC[0][0];
    dX[SV_CEI] = dC[0][1];
    dX[SV_CII] = dC[1][1];
    /* eq. (3) in AdEx form: the subthreshold term is a conductance times a
       voltage, divided by tau_w to be a rate of change of current */
    dX[SV_WE] = -X[SV_WE] / m->tau_w_e + b_e * E + a_e * (tf[0].muV - m->E_L_e) / m->tau_w_e;
    dX[SV_WI] = -X[SV_WI] / m->tau_w_i + m->b_i * I + m->a_i * (tf[1].muV - m->E_L_i) / m->tau_w_i;
    /* eq. (4) with mu = 0; the Wiener increment enters in the stepper */
    dX[SV_OU] = -X[SV_OU] / m->tau_OU;
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller normals.  */
/* ------------------------------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Standard normal for time step n of region k of instance inst: Philox with
   key (seed, inst) and counter (n / 4, k, 0, 0) gives four words; words are
   mapped to (0, 1) as (w + 1/2) 2^-32; pairs (w0, w1), (w2, w3) give two
   Box-Muller pairs (cos, sin); step n takes normal number n mod 4. */
double oracle_normal(uint32_t seed, uint32_t inst, uint64_t n, uint32_t k)
{
    uint32_t ctr[4] = {(uint32_t)(n >> 2), k, 0u, 0u}, key[2] = {seed, inst}, w[4];
    oracle_philox4x32_10(ctr, key, w);
    int q = (int)(n & 3u);
    int pair = q >> 1;
    double u0 = ((double)w[2 * pair] + 0.5) * 0x1p-32;
    double u1 = ((double)w[2 * pair + 1] + 0.5) * 0x1p-32;
    double r = sqrt(-2.0 * log(u0));
    double ang = 2.0 * M_PI * u1;
    return (q & 1) ? r * sin(ang) : r * cos(ang);
}

/* ------------------------------------------------------------------------- */
/* Connectome preparation.                                                    */
/* ------------------------------------------------------------------------- */
/* Row normalisation: W_kj = w_kj / sum_j w_kj; an all-zero row stays zero. */
void oracle_normalise_rows(int n, const double *w, double *W)
{
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += w[k * n + j];
        for (int j = 0; j < n; ++j) W[k * n + j] = s > 0.0 ? w[k * n + j] / s : 0.0;
    }
}

/* Delay in steps: round-half-even(L / (v dt)), at least 1. v (m/s = mm/ms) is
   the single-precision speed the instance was given. */
void oracle_delays(int n, const double *L, float v, double dt, int32_t *d)
{
    for (int i = 0; i < n * n; ++i) {
        double q = nearbyint(L[i] / ((double)v * dt));
        d[i] = q < 1.0 ? 1 : (int32_t)q;
    }
}

/* ------------------------------------------------------------------------- */
/* Pearson FC and summary statistics of one instance.                          */
/* ------------------------------------------------------------------------- */
enum { FLAG_NONFINITE = 1u, FLAG_CLAMP = 2u, FLAG_ZERO_VAR = 4u };

/* x: [ns][n] samples (kHz). w_raw: [n][n] raw SC. Outputs fc [n][n] and
   stats = {fc_mean, fc_std, fc_sc_corr, rate_mean_hz, rate_std_hz, sync_index}.
   A region whose temporal standard deviation is below min_std (kHz) is silent:
   its variance and covariances count as zero, its FC entries are zero (one on
   the diagonal) and the zero-variance flag is set. */
uint32_t oracle_fc_stats(int n, int64_t ns, const double *x, const double *w_raw,
                         double min_std, double *fc, double *stats)
{
    uint32_t flags = 0;
    double *mean = calloc((size_t)n, sizeof(double));
    double *cov = calloc((size_t)n * n, sizeof(double));
    for (int64_t s = 0; s < ns; ++s)
        for (int k = 0; k < n; ++k) mean[k] += x[s * n + k];
    for (int k = 0; k < n; ++k) mean[k] = ns > 0 ? mean[k] / (double)ns : 0.0;
    for (int64_t s = 0; s < ns; ++s)
        for (int k = 0; k < n; ++k)
            for (int l = 0; l < n; ++l)
                cov[k * n + l] += (x[s * n + k] - mean[k]) * (x[s * n + l] - mean[l]);
    for (int i = 0; i < n * n; ++i) cov[i] = ns > 0 ? cov[i] / (double)ns : 0.0;
    for (int k = 0; k < n; ++k)
        if (cov[k * n + k] < min_std * min_std)
            for (int l = 0; l < n; ++l) { cov[k * n + l] = 0.0; cov[l * n + k] = 0.0; }
    for (int k = 0; k < n; ++k)
        for (int l = 0; l < n; ++l) {
            double vk = cov[k * n + k], vl = cov[l * n + l];
            if (k == l) fc[k * n + l] = 1.0;
            else if (vk > 0.0 && vl > 0.0) fc[k * n + l] = cov[k * n + l] / sqrt(vk * vl);
            else fc[k * n + l] = 0.0;
        }
    for (int k = 0; k < n; ++k)
        if (!(cov[k * n + k] > 0.0)) flags |= FLAG_ZERO_VAR;
    /* upper-triangle FC moments and correlation with the raw SC */
    double m_fc = 0, m_w = 0, cnt = 0;
    for (int k = 0; k < n; ++k)
        for (int l = k + 1; l < n; ++l) { m_fc += fc[k * n + l]; m_w += w_raw[k * n + l]; cnt += 1; }
    m_fc = cnt > 0 ? m_fc / cnt : 0.0;
    m_w = cnt > 0 ? m_w / cnt : 0.0;
    double v_fc = 0, v_w = 0, c_fw = 0;
    for (int k = 0; k < n; ++k)
        for (int l = k + 1; l < n; ++l) {
            double a = fc[k * n + l] - m_fc, b = w_raw[k * n + l] - m_w;
            v_fc += a * a; v_w += b * b; c_fw += a * b;
        }
    stats[0] = m_fc;
    stats[1] = cnt > 0 ? sqrt(v_fc / cnt) : 0.0;
    stats[2] = (v_fc > 0 && v_w > 0) ? c_fw / sqrt(v_fc * v_w) : 0.0;
    /* rates in Hz */
    double rm = 0, rs = 0, tot = 0, diag = 0;
    for (int k = 0; k < n; ++k) {
        rm += mean[k];
        rs += sqrt(cov[k * n + k]);
        diag += cov[k * n + k];
        for (int l = 0; l < n; ++l) tot += cov[k * n + l];
    }
    stats[3] = 1000.0 * rm / n;
    stats[4] = 1000.0 * rs / n;
    /* Golomb synchrony: variance of the population mean over mean variance */
    stats[5] = diag > 0 ? sqrt((tot / ((double)n * n)) / (diag / n)) : 0.0;
    free(mean);
    free(cov);
    return flags;
}

/* ------------------------------------------------------------------------- */
/* One Heun step of one region given its coupling input c and normal z.       */
/* ------------------------------------------------------------------------- */
/* Admissible-state projection after each stage. Rates are bounded to
   [0, rate_max]. A rate confined to [0, r] with mean nu has variance at most
   nu (r - nu) (Bhatia-Davis), so each variance is bounded to that range, and
   the cross-covariance by the Cauchy-Schwarz bound sqrt(C_ee C_ii). */
static double clampd(double x, double lo, double hi, uint32_t *hit)
{
    if (x < lo) { *hit = FLAG_CLAMP; return lo; }
    if (x > hi) { *hit = FLAG_CLAMP; return hi; }
    return x;
}
static uint32_t clamp_rates(const or_model *m, double *X)
{
    uint32_t hit = 0;
    const double r = m->rate_max;
    X[SV_E] = clampd(X[SV_E], 0.0, r, &hit);
    X[SV_I] = clampd(X[SV_I], 0.0, r, &hit);
    X[SV_CEE] = clampd(X[SV_CEE], 0.0, X[SV_E] * (r - X[SV_E]), &hit);
    X[SV_CII] = clampd(X[SV_CII], 0.0, X[SV_I] * (r - X[SV_I]), &hit);
    const double cb = sqrt(X[SV_CEE] * X[SV_CII]);
    X[SV_CEI] = clampd(X[SV_CEI], -cb, cb, &hit);
    return hit;
}

/* Python entry: the admissible-state projection on its own (X: 8 states,
   modified in place); returns FLAG_CLAMP when a value moved. */
uint32_t oracle_project(const or_model *m, double *X) { return clamp_rates(m, X); }

/* integrator: 0 = stochastic Heun, 1 = Euler-Maruyama. Returns flag bits. */
uint32_t oracle_step_region(const or_model *m, int integrator, double dt, double *X, double c,
                            double b_e, double a_e, double z)
{
    double f0[N_SV], f1[N_SV], Xt[N_SV];
    uint32_t flags = 0;
    const double gdw = (m->sigma_OU / m->tau_OU) * sqrt(dt) * z;
    oracle_drift(m, X, c, b_e, a_e, f0);
    if (integrator == 1) {
        for (int q = 0; q < N_SV; ++q) X[q] += dt * f0[q];
        X[SV_OU] += gdw;
        return clamp_rates(m, X);
    }
    for (int q = 0; q < N_SV; ++q) Xt[q] = X[q] + dt * f0[q];
    Xt[SV_OU] += gdw;
    flags |= clamp_rates(m, Xt);
    oracle_drift(m, Xt, c, b_e, a_e, f1);
    for (int q = 0; q < N_SV; ++q) X[q] += 0.5 * dt * (f0[q] + f1[q]);
    X[SV_OU] += gdw;
    flags |= clamp_rates(m, X);
    return flags;
}

/* ------------------------------------------------------------------------- */
/* Whole runs.                                                                */
/* ------------------------------------------------------------------------- */
typedef struct {
    double dt;
    int64_t n_steps, transient_steps, tavg_steps, n_trace_steps;
    uint32_t seed;
    int32_t integrator;
    int32_t noise_off; /* 1: z = 0 (deterministic runs for pins) */
    double fc_min_std; /* silence threshold of the FC (kHz) */
} or_run;

typedef struct {
    const or_model *m;
    const or_run *r;
    int n;                 /* regions */
    const double *w_raw;   /* [n][n] */
    const double *L;       /* [n][n] */
    const float *S, *b_e, *a_e, *v;
    const uint32_t *inst_id;
    int64_t n_inst;
    /* outputs, per instance */
    double *final_state;   /* [inst][8][n] */
    double *samples;       /* [inst][ns][n] or NULL */
    double *trace;         /* [inst][n_trace][8][n] or NULL */
    double *fc;            /* [inst][n][n] or NULL */
    double *stats;         /* [inst][6] or NULL */
    uint32_t *flags;       /* [inst] */
    const double *init_state; /* [8] or NULL: uniform initial state override */
    const double *extra;   /* [inst][6] or NULL: per-instance w_noise, tau_w_e, cF_ee, cF_ei,
                              cF_ie, cF_ii (the further sweep axes of Table 4) */
    int64_t next;
    pthread_mutex_t mu;
} run_job;

static void run_instance(run_job *J, int64_t q)
{
    or_model mi = *J->m;   /* the model with this instance's parameters */
    if (J->extra) {
        const double *e = J->extra + q * 6;
        mi.w_noise = e[0];
        mi.tau_w_e = e[1];
        mi.cF_ee = e[2];
        mi.cF_ei = e[3];
        mi.cF_ie = e[4];
        mi.cF_ii = e[5];
    }
    const or_model *m = &mi;
    const or_run *r = J->r;
    const int n = J->n;
    const int64_t ns = (r->n_steps - r->transient_steps) / r->tavg_steps;
    double *W = malloc(sizeof(double) * n * n);
    int32_t *d = malloc(sizeof(int32_t) * n * n);
    double *H = malloc(sizeof(double) * (size_t)(r->n_steps + 1) * n); /* H[m][k], m = 0..n_steps */
    double *X = malloc(sizeof(double) * N_SV * n);
    double *acc = calloc((size_t)n, sizeof(double));
    double *smp = malloc(sizeof(double) * (size_t)(ns > 0 ? ns : 1) * n);
    uint32_t flags = 0;
    oracle_normalise_rows(n, J->w_raw, W);
    oracle_delays(n, J->L, J->v[q], r->dt, d);
    const double S = J->S[q], b_e = J->b_e[q], a_e = J->a_e[q];
    const uint32_t id = J->inst_id[q];
    for (int k = 0; k < n; ++k) {
        double x0[N_SV] = {m->E_init, m->I_init, 0, 0, 0, 0, 0, 0};
        if (J->init_state) memcpy(x0, J->init_state, sizeof(x0));
        for (int s = 0; s < N_SV; ++s) X[s * n + k] = x0[s];
        H[k] = x0[SV_E];
    }
    for (int64_t step = 0; step < r->n_steps; ++step) {
        for (int k = 0; k < n; ++k) {
            /* delayed linear coupling; history before t=0 is the initial rate */
            double c = 0.0;
            for (int j = 0; j < n; ++j) {
                if (W[k * n + j] == 0.0) continue;
                int64_t mt = step - d[k * n + j];
                double h = mt >= 0 ? H[mt * n + j] : H[j];
                c += W[k * n + j] * h;
            }
            c *= S;
            double z = r->noise_off ? 0.0 : oracle_normal(r->seed, id, (uint64_t)step, (uint32_t)k);
            double xs[N_SV];
            for (int s = 0; s < N_SV; ++s) xs[s] = X[s * n + k];
            flags |= oracle_step_region(m, r->integrator, r->dt, xs, c, b_e, a_e, z);
            for (int s = 0; s < N_SV; ++s) {
                if (!isfinite(xs[s])) flags |= FLAG_NONFINITE;
                X[s * n + k] = xs[s];
            }
        }
        for (int k = 0; k < n; ++k) H[(step + 1) * n + k] = X[SV_E * n + k];
        if (J->trace && step < r->n_trace_steps) {
            double *tr = J->trace + ((size_t)q * r->n_trace_steps + step) * N_SV * n;
            memcpy(tr, X, sizeof(double) * N_SV * n);
        }
        /* time average of E over tavg_steps consecutive steps */
        for (int k = 0; k < n; ++k) acc[k] += X[SV_E * n + k];
        if ((step + 1) % r->tavg_steps == 0) {
            int64_t s = (step + 1) / r->tavg_steps - 1 - r->transient_steps / r->tavg_steps;
            for (int k = 0; k < n; ++k) {
                if (s >= 0 && s < ns) smp[s * n + k] = acc[k] / (double)r->tavg_steps;
                acc[k] = 0.0;
            }
        }
    }
    memcpy(J->final_state + (size_t)q * N_SV * n, X, sizeof(double) * N_SV * n);
    if (J->samples && ns > 0) memcpy(J->samples + (size_t)q * ns * n, smp, sizeof(double) * ns * n);
    if (J->fc || J->stats) {
        double *fc = J->fc ? J->fc + (size_t)q * n * n : malloc(sizeof(double) * n * n);
        double st[6];
        flags |= oracle_fc_stats(n, ns, smp, J->w_raw, r->fc_min_std, fc, st);
        if (J->stats) memcpy(J->stats + q * 6, st, sizeof(st));
        if (!J->fc) free(fc);
    }
    J->flags[q] = flags;
    free(W); free(d); free(H); free(X); free(acc); free(smp);
}

static void *run_worker(void *arg)
{
    run_job *J = arg;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        int64_t q = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (q >= J->n_inst) break;
        run_instance(J, q);
    }
    return NULL;
}

/* Re-anchored steps of one instance: for every step n < n_steps, the oracle's
   step n taken from a given state -- trace_in[n-1] (the state after step
   n-1), or the initial state for n = 0 -- with the coupling formed from the
   given excitatory-rate history (E of trace_in; the initial rate before the
   first step) and the instance's own Philox normal of step n. out[n] is the
   state after that one step, to compare with trace_in[n]: each step of
   another implementation is checked on its own, whatever the trajectory's
   sensitivity to earlier rounding. trace_in, out: [n_steps][8][n]. extra:
   NULL or the six further per-instance parameters (as in oracle_run).
   Returns the OR of the step flags. */
uint32_t oracle_anchored_steps(const or_model *m0, const or_run *r, int n, const double *w_raw,
                               const double *L, float S, float b_e, float a_e, float v,
                               uint32_t inst_id, const double *extra, int64_t n_steps,
                               const double *trace_in, double *out)
{
    or_model mi = *m0;
    if (extra) {
        mi.w_noise = extra[0]; mi.tau_w_e = extra[1];
        mi.cF_ee = extra[2]; mi.cF_ei = extra[3]; mi.cF_ie = extra[4]; mi.cF_ii = extra[5];
    }
    const or_model *m = &mi;
    double *W = malloc(sizeof(double) * n * n);
    int32_t *d = malloc(sizeof(int32_t) * n * n);
    uint32_t flags = 0;
    oracle_normalise_rows(n, w_raw, W);
    oracle_delays(n, L, v, r->dt, d);
    for (int64_t step = 0; step < n_steps; ++step) {
        for (int k = 0; k < n; ++k) {
            double c = 0.0;
            for (int j = 0; j < n; ++j) {
                if (W[k * n + j] == 0.0) continue;
                /* history value at step mt: E after step mt-1, initial before */
                int64_t mt = step - d[k * n + j];
                double h = mt >= 1 ? trace_in[((size_t)(mt - 1) * N_SV + SV_E) * n + j] : m->E_init;
                c += W[k * n + j] * h;
            }
            c *= S;
            double xs[N_SV];
            for (int q = 0; q < N_SV; ++q) {
                if (step == 0) {
                    double x0[N_SV] = {m->E_init, m->I_init, 0, 0, 0, 0, 0, 0};
                    xs[q] = x0[q];
                } else {
                    xs[q] = trace_in[((size_t)(step - 1) * N_SV + q) * n + k];
                }
            }
            double z = r->noise_off ? 0.0 : oracle_normal(r->seed, inst_id, (uint64_t)step, (uint32_t)k);
            flags |= oracle_step_region(m, r->integrator, r->dt, xs, c, b_e, a_e, z);
            for (int q = 0; q < N_SV; ++q) out[((size_t)step * N_SV + q) * n + k] = xs[q];
        }
    }
    free(W);
    free(d);
    return flags;
}

/* Runs n_inst instances on one connectome with n_threads threads (one
   instance per thread at a time). Any output pointer may be NULL except
   final_state and flags. */
int oracle_run(const or_model *m, const or_run *r, int n, const double *w_raw, const double *L,
               int64_t n_inst, const float *S, const float *b_e, const float *a_e, const float *v,
               const uint32_t *inst_id, const double *init_state, const double *extra,
               double *final_state,
               double *samples, double *trace, double *fc, double *stats, uint32_t *flags,
               int n_threads)
{
    if (n <= 0 || n_inst < 0 || r->tavg_steps <= 0 || r->n_steps < 0) return -1;
    run_job J;
    memset(&J, 0, sizeof(J));
    J.m = m; J.r = r; J.n = n; J.w_raw = w_raw; J.L = L;
    J.S = S; J.b_e = b_e; J.a_e = a_e; J.v = v; J.inst_id = inst_id; J.n_inst = n_inst;
    J.final_state = final_state; J.samples = samples; J.trace = trace; J.fc = fc;
    J.stats = stats; J.flags = flags; J.init_state = init_state; J.extra = extra;
    pthread_mutex_init(&J.mu, NULL);
    if (n_threads < 1) n_threads = 1;
    pthread_t *th = malloc(sizeof(pthread_t) * n_threads);
    for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, run_worker, &J);
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&J.mu);
    return 0;
}
