// adex_model.h -- single-precision TVB-AdEx mean-field step for the GPU.
//
// Everything here is templated on the scalar type T so the same arithmetic can
// be instantiated on the host with an operation-counting type; on the device T
// is float and the scalar primitives map to CDNA4 VALU instructions.
//
// Transfer function (Section 2.2): inputs xe, xi (kHz), adaptation W (pA).
// Mean conductances ge = Q_e tau_e K_e xe, gi = Q_i tau_i K_i xi, total
// G = g_L + ge + gi; mean voltage mu_V = (ge E_e + gi E_i + g_L E_L - W)/G;
// PSP amplitudes U_s = Q_s (E_s - mu_V)/G; shot-noise weights
// A_s = K_s x_s (tau_s U_s)^2; with T_eff = C_m/G and d_s = 1/(T_eff + tau_s):
// sigma_V^2 = (A_e d_e + A_i d_i)/2, tau_V = (A_e + A_i)/(A_e d_e + A_i d_i),
// tau_N = tau_V g_L/C_m; threshold = quadratic polynomial (Table 1) of the
// normalised (mu_V, sigma_V, tau_N); F = erfc((V_thre - mu_V)/(sqrt2 sigma_V))
// / (2 tau_V). The value and the exact first and second derivatives in
// (xe, xi) are carried as 6-component jets; the derivatives of every quantity
// that depends on the inputs only through G are formed from its scalar
// derivatives in G, and mu_V's derivatives from its closed form.
//
// Drift (Section 2.1, eq. 1-3) and OU (eq. 4): see step_region().
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define VADX_HD __host__ __device__ __forceinline__
#else
#define VADX_HD inline
#endif

namespace vadx {

// FP32 constants of the model, derived on the host from vadx_model.
struct KModel {
    float aE, aI;               // Q_e tau_e K_e, Q_i tau_i K_i  (nS per kHz)
    float gL, Cm, Ee, Ei, Qe, Qi, tau_e, tau_i;
    float KeTe2, KiTi2;         // K_e tau_e^2, K_i tau_i^2
    float EL[2];                // E_L for pop 0 (exc), 1 (inh)
    float gLEL[2];              // g_L E_L
    float P[2][10];             // threshold polynomial coefficients (Table 1 order)
    float mu_s, mu_o;           // m = mu_V * mu_s + mu_o
    float sg_s, sg_o;           // s = sigma_V * sg_s + sg_o
    float tn_s, tn_o;           // t = tau_V * tn_s + tn_o
    float invT, invNe, invNi;
    float inv_tauw[2], b_i, a_i;
    float cF[2][2];             // cF[pop][0 = exc input, 1 = inh input]
    float inv_tauOU, ou_gain;   // 1/tau_OU, sigma_OU / tau_OU
    float w_noise, rate_max, x_floor;
    float E_init, I_init;
};

// A value with its gradient (a = d/dxe, b = d/dxi) and Hessian.
template <class T> struct Jet { T v, a, b, aa, ab, bb; };

// ---------------------------------------------------------------- primitives
// The scalar primitives a type must provide (float overloads below):
//   rcp(x) = 1/x, rsq(x) = 1/sqrt(x), sqr(x) = sqrt(x), ex2(x) = 2^x,
//   lg2(x) = log2(x), fma(a, b, c) = a*b + c.
VADX_HD float rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
VADX_HD float rsq(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.0f / __builtin_sqrtf(x);
#endif
}
VADX_HD float sqr(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return __builtin_sqrtf(x);
#endif
}
VADX_HD float ex2(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_exp2f(x);
#else
    return __builtin_exp2f(x);
#endif
}
VADX_HD float lg2(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_logf(x);
#else
    return __builtin_log2f(x);
#endif
}
VADX_HD double sqr(double x) { return __builtin_sqrt(x); }
VADX_HD float fmaf_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
VADX_HD float absf_(float x) { return __builtin_fabsf(x); }
VADX_HD float selectf(bool c, float a, float b) { return c ? a : b; }
VADX_HD float maxf_(float a, float b) { return __builtin_fmaxf(a, b); }

// ---------------------------------------------------------------- jet algebra
template <class T> VADX_HD Jet<T> jmul(const Jet<T> &x, const Jet<T> &y)
{
    Jet<T> r;
    r.v = x.v * y.v;
    r.a = fmaf_(x.a, y.v, x.v * y.a);
    r.b = fmaf_(x.b, y.v, x.v * y.b);
    r.aa = fmaf_(x.aa, y.v, fmaf_(T(2) * x.a, y.a, x.v * y.aa));
    r.ab = fmaf_(x.ab, y.v, fmaf_(x.a, y.b, fmaf_(x.b, y.a, x.v * y.ab)));
    r.bb = fmaf_(x.bb, y.v, fmaf_(T(2) * x.b, y.b, x.v * y.bb));
    return r;
}
template <class T> VADX_HD Jet<T> jsq(const Jet<T> &x)
{
    Jet<T> r;
    T v2 = T(2) * x.v;
    r.v = x.v * x.v;
    r.a = v2 * x.a;
    r.b = v2 * x.b;
    r.aa = fmaf_(v2, x.aa, T(2) * x.a * x.a);
    r.ab = fmaf_(v2, x.ab, T(2) * x.a * x.b);
    r.bb = fmaf_(v2, x.bb, T(2) * x.b * x.b);
    return r;
}
template <class T> VADX_HD Jet<T> jadd(const Jet<T> &x, const Jet<T> &y)
{
    return Jet<T>{x.v + y.v, x.a + y.a, x.b + y.b, x.aa + y.aa, x.ab + y.ab, x.bb + y.bb};
}
// s*x + c
template <class T> VADX_HD Jet<T> jaffine(const Jet<T> &x, T s, T c)
{
    return Jet<T>{fmaf_(s, x.v, c), s * x.a, s * x.b, s * x.aa, s * x.ab, s * x.bb};
}
// f(x) given f, f', f'' at x.v (chain rule to second order)
template <class T> VADX_HD Jet<T> jchain(const Jet<T> &x, T f0, T f1, T f2)
{
    Jet<T> r;
    r.v = f0;
    r.a = f1 * x.a;
    r.b = f1 * x.b;
    T fa = f2 * x.a;
    r.aa = fmaf_(f1, x.aa, fa * x.a);
    r.ab = fmaf_(f1, x.ab, fa * x.b);
    r.bb = fmaf_(f1, x.bb, f2 * x.b * x.b);
    return r;
}
// a function of G = g_L + aE xe + aI xi only: f, f', f'' in G
template <class T> VADX_HD Jet<T> jofG(T f0, T f1, T f2, T aE, T aI)
{
    T f2e = f2 * aE;
    return Jet<T>{f0, f1 * aE, f1 * aI, f2e * aE, f2e * aI, f2 * aI * aI};
}

// erfc with a shared exp(-z^2): Numerical Recipes' Chebyshev fit
// erfc(|z|) = t exp(-z^2 + p(t)), t = 1/(1 + |z|/2), fractional error < 1.2e-7
// (Press et al., Numerical Recipes, section 6.2). Returns erfc(z) and
// e = exp(-z^2) (for the derivatives).
template <class T> VADX_HD void erfc_and_gauss(T z, T &g, T &e)
{
    const T L2E = T(1.4426950408889634f);
    T az = absf_(z);
    T t = rcp(fmaf_(T(0.5f), az, T(1.0f)));
    T p = fmaf_(t, T(0.17087277f), T(-0.82215223f));
    p = fmaf_(t, p, T(1.48851587f));
    p = fmaf_(t, p, T(-1.13520398f));
    p = fmaf_(t, p, T(0.27886807f));
    p = fmaf_(t, p, T(-0.18628806f));
    p = fmaf_(t, p, T(0.09678418f));
    p = fmaf_(t, p, T(0.37409196f));
    p = fmaf_(t, p, T(1.00002368f));
    p = fmaf_(t, p, T(-1.26551223f));
    T z2 = az * az;
    e = ex2(-z2 * L2E);
    T g_pos = t * e * ex2(p * L2E);
    g = selectf(z >= T(0), g_pos, T(2) - g_pos);
}

// Transfer function of population `pop` with its value and derivatives in
// (xe, xi). Also returns mu_V (value) for the adaptation equation.
// EQ: tau_e == tau_i, so d_i = d_e, 1/tau_V = d_e and sigma_V^2 = (A_e + A_i) d_e / 2.
template <bool EQ, class T>
VADX_HD Jet<T> transfer(const KModel &M, int pop, T xe, T xi, T W, T &muV_out)
{
    const T aE = T(M.aE), aI = T(M.aI);
    T ge = aE * xe, gi = aI * xi;
    T G = T(M.gL) + ge + gi;
    T r = rcp(G);
    // 1/G as a jet: (1/G)' = -r^2, (1/G)'' = 2 r^3
    T r2 = r * r;
    Jet<T> R = jofG(r, -r2, T(2) * r2 * r, aE, aI);
    // mu_V and its closed-form derivatives
    T mu = fmaf_(ge, T(M.Ee), fmaf_(gi, T(M.Ei), T(M.gLEL[pop]) - W)) * r;
    T dEe = T(M.Ee) - mu, dEi = T(M.Ei) - mu;
    T mu_a = aE * dEe * r, mu_b = aI * dEi * r;
    Jet<T> MU;
    MU.v = mu;
    MU.a = mu_a;
    MU.b = mu_b;
    MU.aa = T(-2) * aE * r * mu_a;
    MU.ab = -r * fmaf_(aE, mu_b, aI * mu_a);
    MU.bb = T(-2) * aI * r * mu_b;
    muV_out = mu;
    // PSP amplitudes U_s = Q_s (E_s - mu_V) / G
    Jet<T> dE{dEe, -MU.a, -MU.b, -MU.aa, -MU.ab, -MU.bb};
    Jet<T> dI{dEi, -MU.a, -MU.b, -MU.aa, -MU.ab, -MU.bb};
    Jet<T> Ue2 = jsq(jmul(dE, R));   // (U_e / Q_e)^2
    Jet<T> Ui2 = jsq(jmul(dI, R));   // (U_i / Q_i)^2
    // A_e = K_e tau_e^2 Q_e^2 xe (U_e/Q_e)^2: times a function linear in xe
    const T ce = T(M.KeTe2) * T(M.Qe) * T(M.Qe), ci = T(M.KiTi2) * T(M.Qi) * T(M.Qi);
    T lxe = ce * xe, lxi = ci * xi;
    Jet<T> Ae{lxe * Ue2.v, fmaf_(ce, Ue2.v, lxe * Ue2.a), lxe * Ue2.b,
              fmaf_(T(2) * ce, Ue2.a, lxe * Ue2.aa), fmaf_(ce, Ue2.b, lxe * Ue2.ab),
              lxe * Ue2.bb};
    Jet<T> Ai{lxi * Ui2.v, lxi * Ui2.a, fmaf_(ci, Ui2.v, lxi * Ui2.b), lxi * Ui2.aa,
              fmaf_(ci, Ui2.a, lxi * Ui2.ab), fmaf_(T(2) * ci, Ui2.b, lxi * Ui2.bb)};
    // d_s = 1/(C_m/G + tau_s) = G/(C_m + tau_s G): h' = C_m (d r)^2, h'' = -2 tau_s C_m (d r)^3
    T de = rcp(fmaf_(T(M.Cm), r, T(M.tau_e)));
    T qe = de * r;
    T he1 = T(M.Cm) * qe * qe;
    const T he2 = T(-2) * T(M.tau_e) * he1 * qe;
    Jet<T> De = jofG(de, he1, he2, aE, aI);
    Jet<T> As = jadd(Ae, Ai);
    Jet<T> S2, ITV, TV;                              // 2 sigma_V^2, 1/tau_V, tau_V
    if constexpr (EQ) {
        S2 = jmul(As, De);
        ITV = De;
        // tau_V = T_eff + tau_e = C_m/G + tau_e
        TV = jofG(fmaf_(T(M.Cm), r, T(M.tau_e)), -T(M.Cm) * r2, T(2) * T(M.Cm) * r2 * r, aE, aI);
    } else {
        T di = rcp(fmaf_(T(M.Cm), r, T(M.tau_i)));
        T qi = di * r;
        T hi1 = T(M.Cm) * qi * qi;
        const T hi2 = T(-2) * T(M.tau_i) * hi1 * qi;
        Jet<T> Di = jofG(di, hi1, hi2, aE, aI);
        S2 = jadd(jmul(Ae, De), jmul(Ai, Di));
        // 1/tau_V = (A_e d_e + A_i d_i)/(A_e + A_i) = d_e + w (d_i - d_e) with
        // w = A_i/(A_e + A_i): a weighted mean of d_e, d_i whose derivatives do
        // not cancel when one source dominates (the ratio form loses them in FP32).
        T ra = rcp(As.v);
        T ra2 = ra * ra;
        Jet<T> RA = jchain(As, ra, -ra2, T(2) * ra2 * ra);
        Jet<T> Wi = jmul(Ai, RA);
        Jet<T> Dd = jofG(di - de, hi1 - he1, hi2 - he2, aE, aI);
        ITV = jadd(De, jmul(Wi, Dd));
        T itv = rcp(ITV.v);
        T itv2 = itv * itv;
        TV = jchain(ITV, itv, -itv2, T(2) * itv2 * itv);
    }
    // q = S2^(-1/2) = 1/(sqrt2 sigma_V);  (x^-1/2)' = -q^3/2, '' = 3 q^5/4
    T q = rsq(S2.v);
    T q2 = q * q, q3 = q2 * q;
    Jet<T> Q = jchain(S2, q, T(-0.5f) * q3, T(0.75f) * q3 * q2);
    // sigma_V = S2 q / sqrt2
    Jet<T> SQ = jmul(S2, Q);
    // normalised polynomial coordinates
    Jet<T> mm = jaffine(MU, T(M.mu_s), T(M.mu_o));
    Jet<T> ss = jaffine(SQ, T(M.sg_s), T(M.sg_o));   // sg_s includes 1/sqrt2
    Jet<T> tt = jaffine(TV, T(M.tn_s), T(M.tn_o));
    const float *P = M.P[pop];
    // V_thre - mu_V = P0 + m (P1 + P4 m + P7 s + P8 t) + s (P2 + P5 s + P9 t)
    //                 + t (P3 + P6 t) - mu_V
    Jet<T> c1 = jaffine(mm, T(P[4]), T(P[1]));
    c1 = jadd(c1, jaffine(ss, T(P[7]), T(0)));
    c1 = jadd(c1, jaffine(tt, T(P[8]), T(0)));
    Jet<T> c2 = jaffine(ss, T(P[5]), T(P[2]));
    c2 = jadd(c2, jaffine(tt, T(P[9]), T(0)));
    Jet<T> c3 = jaffine(tt, T(P[6]), T(P[3]));
    Jet<T> V = jadd(jadd(jmul(mm, c1), jmul(ss, c2)), jmul(tt, c3));
    V = jadd(V, jaffine(MU, T(-1), T(P[0])));
    Jet<T> Z = jmul(V, Q);                            // (V_thre - mu_V)/(sqrt2 sigma_V)
    T g, e;
    erfc_and_gauss(Z.v, g, e);
    const T TWO_OVER_SQRTPI = T(1.1283791670955126f);
    T g1 = -TWO_OVER_SQRTPI * e;
    Jet<T> GZ = jchain(Z, g, g1, T(-2) * Z.v * g1);
    Jet<T> F = jmul(GZ, ITV);
    return jaffine(F, T(0.5f), T(0));
}

// Per-instance parameters.
template <class T> struct InstParams { T S, b_e, a_e; };

// Drift of one region's 8 states given its coupling input c (eq. 1-4).
template <bool EQ, class T>
VADX_HD void drift(const KModel &M, const T X[8], T c, T be, T ae, T dX[8])
{
    const T E = X[0], I = X[1], Cee = X[2], Cei = X[3], Cii = X[4];
    T exc = E + c + T(M.w_noise) * X[7];
    T xe0 = maxf_(exc + T(M.cF[0][0]), T(M.x_floor));
    T xi0 = maxf_(I + T(M.cF[0][1]), T(M.x_floor));
    T xe1 = maxf_(exc + T(M.cF[1][0]), T(M.x_floor));
    T xi1 = maxf_(I + T(M.cF[1][1]), T(M.x_floor));
    T muVe, muVi;
    Jet<T> Fe = transfer<EQ>(M, 0, xe0, xi0, X[5], muVe);
    Jet<T> Fi = transfer<EQ>(M, 1, xe1, xi1, X[6], muVi);
    const T iT = T(M.invT);
    T fe = Fe.v - E, fi = Fi.v - I;
    // eq. 1: T dnu/dt = (F - nu) + 1/2 C_ee F_ee + C_ei F_ei + 1/2 C_ii F_ii
    dX[0] = iT * fmaf_(T(0.5f), fmaf_(Cee, Fe.aa, Cii * Fe.bb), fmaf_(Cei, Fe.ab, fe));
    dX[1] = iT * fmaf_(T(0.5f), fmaf_(Cee, Fi.aa, Cii * Fi.bb), fmaf_(Cei, Fi.ab, fi));
    // eq. 2
    dX[2] = iT * fmaf_(Fe.v * (iT - Fe.v), T(M.invNe),
                       fmaf_(fe, fe, T(2) * (fmaf_(Cee, Fe.a, Cei * Fe.b) - Cee)));
    dX[3] = iT * fmaf_(fe, fi, fmaf_(Cee, Fi.a, fmaf_(Cei, Fi.b + Fe.a,
                                                        fmaf_(Cii, Fe.b, T(-2) * Cei))));
    dX[4] = iT * fmaf_(Fi.v * (iT - Fi.v), T(M.invNi),
                       fmaf_(fi, fi, T(2) * (fmaf_(Cii, Fi.b, Cei * Fi.a) - Cii)));
    // eq. 3 (AdEx form, subthreshold term over tau_w)
    dX[5] = fmaf_(be, E, T(M.inv_tauw[0]) * fmaf_(ae, muVe - T(M.EL[0]), -X[5]));
    dX[6] = fmaf_(T(M.b_i), I, T(M.inv_tauw[1]) * fmaf_(T(M.a_i), muVi - T(M.EL[1]), -X[6]));
    // eq. 4, deterministic part
    dX[7] = -X[7] * T(M.inv_tauOU);
}

// Projection onto admissible states after each stage: rates in [0, rate_max],
// variances in [0, nu (rate_max - nu)] (bound for a variable confined to
// [0, rate_max] with mean nu), |C_ei| <= sqrt(C_ee C_ii). Comparisons are
// written so that a NaN passes through. Returns true when a bound was hit.
template <class T> VADX_HD T clampv(T x, T lo, T hi, bool &hit)
{
    bool l = x < lo, h = x > hi;
    hit = hit || l || h;
    return l ? lo : (h ? hi : x);
}
template <class T> VADX_HD bool project(const KModel &M, T X[8])
{
    bool hit = false;
    const T rm = T(M.rate_max);
    X[0] = clampv(X[0], T(0), rm, hit);
    X[1] = clampv(X[1], T(0), rm, hit);
    X[2] = clampv(X[2], T(0), X[0] * (rm - X[0]), hit);
    X[4] = clampv(X[4], T(0), X[1] * (rm - X[1]), hit);
    T cb = sqr(X[2] * X[4]);
    X[3] = clampv(X[3], -cb, cb, hit);
    return hit;
}

// One step of stochastic Heun (or Euler-Maruyama) for one region. The drift
// is evaluated in T (float); the state X and its increments are accumulated
// in S (double), so the rounding of the state does not build up over the
// run. gdw is the OU increment (sigma/tau_OU) sqrt(dt) z. Returns true when a
// bound was hit.
template <bool EQ, class T, class S>
VADX_HD bool step_region(const KModel &M, int integrator, S dt, S X[8], T c, T be, T ae, S gdw)
{
    T xf[8], f0[8], f1[8];
    S Xt[8];
    for (int q = 0; q < 8; ++q) xf[q] = T(X[q]);
    drift<EQ>(M, xf, c, be, ae, f0);
    if (integrator == 1) {
        for (int q = 0; q < 8; ++q) X[q] = X[q] + dt * S(f0[q]);
        X[7] = X[7] + gdw;
        return project(M, X);
    }
    for (int q = 0; q < 8; ++q) Xt[q] = X[q] + dt * S(f0[q]);
    Xt[7] = Xt[7] + gdw;
    bool hit = project(M, Xt);
    for (int q = 0; q < 8; ++q) xf[q] = T(Xt[q]);
    drift<EQ>(M, xf, c, be, ae, f1);
    const S hdt = S(0.5) * dt;
    for (int q = 0; q < 8; ++q) X[q] = X[q] + hdt * (S(f0[q]) + S(f1[q]));
    X[7] = X[7] + gdw;
    hit = project(M, X) || hit;
    return hit;
}

} // namespace vadx
