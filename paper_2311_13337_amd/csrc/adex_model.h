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

// FP32 constants of the model, derived on the host from vadx_model
// (make_kmodel in kmodel.h).
struct KModel {
    float aE, aI;               // Q_e tau_e K_e, Q_i tau_i K_i  (nS per kHz)
    float gL, Cm, Ee, Ei, tau_e, tau_i;
    float ce, ci;               // K_e tau_e^2 Q_e^2, K_i tau_i^2 Q_i^2
    float aEE, aEI, aII;        // aE^2, aE aI, aI^2
    float bE, bI;               // aI (E_e - E_i), aE (E_i - E_e)
    float EegL, EigL;           // E_e g_L, E_i g_L
    float ce2bE, ci2bI;         // 2 c_e bE, 2 c_i bI
    float ce2bE2, ci2bI2;       // 2 c_e bE^2, 2 c_i bI^2
    float EL[2];                // E_L for pop 0 (exc), 1 (inh)
    float gLEL[2];              // g_L E_L
    // threshold polynomial (Table 1) in offsets d = u - pc of the raw
    // coordinates u = (mu_V, sqrt2 sigma_V, tau_V) from the centre of their
    // normalisation: P0 + plin . d + d . Hraw d / 2
    float P0[2];
    float plin[2][3];
    float Hraw[2][6];           // 00 01 02 11 12 22
    float pc[3];
    float invT, invNe, invNi;
    float inv_tauw[2], b_i, a_i;
    float cF[2][2];             // cF[pop][0 = exc input, 1 = inh input]
    float inv_tauOU;
    float w_noise, rate_max, x_floor;
    int same_inputs;            // both populations see the same (xe, xi): cF_ee = cF_ie, cF_ei = cF_ii
};

// Model variant of an instantiation of the step: bit 0 when tau_e == tau_i
// (one d_s, tau_V a function of G alone), bit 1 when both populations see the
// same inputs (the G-dependent parts of their transfer functions coincide).
enum { kVarEq = 1, kVarSame = 2 };
inline int model_variant(const KModel &M)
{
    return (M.tau_e == M.tau_i ? kVarEq : 0) | (M.same_inputs ? kVarSame : 0);
}

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
VADX_HD double maxd_(double a, double b) { return __builtin_fmax(a, b); }
VADX_HD double mind_(double a, double b) { return __builtin_fmin(a, b); }
VADX_HD bool finite_(float x) { return __builtin_isfinite(x); }
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

// x * f(G) for f known through f, f', f'' in G (aEE = aE^2, aEI = aE aI, aII = aI^2)
template <class T>
VADX_HD Jet<T> jmulG(const Jet<T> &x, T f0, T f1, T f2, T aE, T aI, T aEE, T aEI, T aII)
{
    T fa = f1 * aE, fb = f1 * aI, v2 = x.v * f2;
    Jet<T> r;
    r.v = x.v * f0;
    r.a = fmaf_(x.a, f0, x.v * fa);
    r.b = fmaf_(x.b, f0, x.v * fb);
    r.aa = fmaf_(x.aa, f0, fmaf_(T(2) * x.a, fa, v2 * aEE));
    r.ab = fmaf_(x.ab, f0, fmaf_(x.a, fb, fmaf_(x.b, fa, v2 * aEI)));
    r.bb = fmaf_(x.bb, f0, fmaf_(T(2) * x.b, fb, v2 * aII));
    return r;
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
// The parts of the transfer function that depend on the inputs only through
// xe, xi and G = g_L + a_e xe + a_i xi, not on the population: shared by the
// two populations when their inputs coincide.
template <class T> struct TFShared {
    T xe, xi, r, r2, r3;
    T de, he1, he2;             // d_e = 1/(C_m/G + tau_e) and its first two derivatives in G
    T cexe, cixi;               // c_e xe, c_i xi
    // tau_e == tau_i only: phi = d_e / G^4 with its derivatives in G, and the
    // jets of 1/tau_V = d_e and tau_V = C_m/G + tau_e
    T phi, phi1, phi2;
    Jet<T> ITV, TV;
};

template <bool EQ, class T> VADX_HD TFShared<T> tf_shared(const KModel &M, T xe, T xi)
{
    TFShared<T> g;
    const T aE = T(M.aE), aI = T(M.aI);
    g.xe = xe;
    g.xi = xi;
    T G = fmaf_(aE, xe, fmaf_(aI, xi, T(M.gL)));
    g.r = rcp(G);
    g.r2 = g.r * g.r;
    g.r3 = g.r2 * g.r;
    // d_s = 1/(C_m/G + tau_s) = G/(C_m + tau_s G): h' = C_m (d r)^2, h'' = -2 tau_s C_m (d r)^3
    g.de = rcp(fmaf_(T(M.Cm), g.r, T(M.tau_e)));
    T qe = g.de * g.r;
    g.he1 = T(M.Cm) * qe * qe;
    g.he2 = T(-2) * T(M.tau_e) * g.he1 * qe;
    g.cexe = T(M.ce) * xe;
    g.cixi = T(M.ci) * xi;
    if constexpr (EQ) {
        // (ln phi)' = -(3 + tau d_e)/G, phi'' = phi (12 + 6 tau d_e + 2 (tau d_e)^2) / G^2
        T td = T(M.tau_e) * g.de;
        g.phi = g.r2 * g.r2 * g.de;
        g.phi1 = -g.phi * g.r * (T(3) + td);
        g.phi2 = g.phi * g.r2 * fmaf_(td, fmaf_(T(2), td, T(6)), T(12));
        g.ITV = jofG(g.de, g.he1, g.he2, aE, aI);
        // tau_V = T_eff + tau_e = C_m/G + tau_e
        g.TV = jofG(fmaf_(T(M.Cm), g.r, T(M.tau_e)), -T(M.Cm) * g.r2, T(2) * T(M.Cm) * g.r3, aE, aI);
    }
    return g;
}

template <bool EQ, class T>
VADX_HD Jet<T> transfer(const KModel &M, int pop, const TFShared<T> &g, T W, T &muV_out)
{
    const T aE = T(M.aE), aI = T(M.aI);
    const T xe = g.xe, xi = g.xi, r = g.r, r2 = g.r2, r3 = g.r3;
    const T de = g.de, he1 = g.he1, he2 = g.he2;
    // mu_V through A = (E_e - mu_V) G = alpha_e + beta_e xi (linear in xi) and
    // B = (E_i - mu_V) G = alpha_i + beta_i xe (linear in xe): mu_V = E_e - A/G
    T c0 = T(M.gLEL[pop]) - W;
    T A = fmaf_(T(M.bE), xi, T(M.EegL) - c0);
    T B = fmaf_(T(M.bI), xe, T(M.EigL) - c0);
    T Ar2 = A * r2, Ar3 = T(2) * A * r3, bEr2 = T(M.bE) * r2;
    Jet<T> MU;
    MU.v = fmaf_(-A, r, T(M.Ee));
    MU.a = Ar2 * aE;
    MU.b = fmaf_(Ar2, aI, -T(M.bE) * r);
    MU.aa = -Ar3 * T(M.aEE);
    MU.ab = fmaf_(bEr2, aE, -Ar3 * T(M.aEI));
    MU.bb = fmaf_(T(2) * bEr2, aI, -Ar3 * T(M.aII));
    muV_out = MU.v;
    // shot-noise weights A_s = K_s x_s (tau_s U_s)^2 with U_e = Q_e A/G^2,
    // U_i = Q_i B/G^2: A_e + A_i = Pi / G^4 with the cubic
    // Pi = c_e xe A^2 + c_i xi B^2 (c_s = K_s tau_s^2 Q_s^2), whose derivatives
    // are exact polynomials
    const T ce = T(M.ce), ci = T(M.ci);
    const T cexe = g.cexe, cixi = g.cixi;
    T A2 = A * A, B2 = B * B;
    Jet<T> PI;
    PI.v = fmaf_(cexe, A2, cixi * B2);
    PI.a = fmaf_(ce, A2, T(M.ci2bI) * xi * B);
    PI.b = fmaf_(T(M.ce2bE) * xe, A, ci * B2);
    PI.aa = T(M.ci2bI2) * xi;
    PI.ab = fmaf_(T(M.ce2bE), A, T(M.ci2bI) * B);
    PI.bb = T(M.ce2bE2) * xe;
    Jet<T> S2, ITV, TV;                              // 2 sigma_V^2, 1/tau_V, tau_V
    if constexpr (EQ) {
        // S2 = Pi phi(G), phi = d_e / G^4
        S2 = jmulG(PI, g.phi, g.phi1, g.phi2, aE, aI, T(M.aEE), T(M.aEI), T(M.aII));
        ITV = g.ITV;
        TV = g.TV;
    } else {
        // A_e = c_e xe A^2 / G^4 and A_i = c_i xi B^2 / G^4 weighted separately
        Jet<T> Ae, Ai;
        Ae.v = cexe * A2; Ae.a = ce * A2; Ae.b = T(M.ce2bE) * xe * A;
        Ae.aa = T(0); Ae.ab = T(M.ce2bE) * A; Ae.bb = T(M.ce2bE2) * xe;
        Ai.v = cixi * B2; Ai.a = T(M.ci2bI) * xi * B; Ai.b = ci * B2;
        Ai.aa = T(M.ci2bI2) * xi; Ai.ab = T(M.ci2bI) * B; Ai.bb = T(0);
        T r4 = r2 * r2;
        Jet<T> R4 = jofG(r4, T(-4) * r4 * r, T(20) * r4 * r2, aE, aI);
        Ae = jmul(Ae, R4);
        Ai = jmul(Ai, R4);
        Jet<T> De = jofG(de, he1, he2, aE, aI);
        T di = rcp(fmaf_(T(M.Cm), r, T(M.tau_i)));
        T qi = di * r;
        T hi1 = T(M.Cm) * qi * qi;
        const T hi2 = T(-2) * T(M.tau_i) * hi1 * qi;
        Jet<T> Di = jofG(di, hi1, hi2, aE, aI);
        S2 = jadd(jmul(Ae, De), jmul(Ai, Di));
        // 1/tau_V = (A_e d_e + A_i d_i)/(A_e + A_i) = d_e + w (d_i - d_e) with
        // w = A_i/(A_e + A_i): a weighted mean of d_e, d_i whose derivatives do
        // not cancel when one source dominates (the ratio form loses them in FP32).
        Jet<T> As = jadd(Ae, Ai);
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
    // SQ = sqrt(S2) = sqrt2 sigma_V;  (x^1/2)' = q/2, '' = -q^3/4
    Jet<T> SQ = jchain(S2, S2.v * q, T(0.5f) * q, T(-0.25f) * q3);
    // V = V_thre - mu_V with the threshold polynomial p of Table 1 written in
    // the offsets d = u - c of u = (mu_V, SQ, tau_V) from the centre c of its
    // normalisation: p = P0 + L.d + d.H d / 2 with L_k = P_k s_k and the constant
    // Hessian H_kl = s_k s_l d2p/dn_k dn_l, so grad p = L + H d and the jet of
    // V follows from the jets of u by the chain rule.
    const float *L = M.plin[pop], *Hr = M.Hraw[pop];
    T d0 = MU.v - T(M.pc[0]), d1 = SQ.v - T(M.pc[1]), d2 = TV.v - T(M.pc[2]);
    T k0 = fmaf_(T(Hr[0]), d0, fmaf_(T(Hr[1]), d1, fmaf_(T(Hr[2]), d2, T(L[0]))));
    T k1 = fmaf_(T(Hr[1]), d0, fmaf_(T(Hr[3]), d1, fmaf_(T(Hr[4]), d2, T(L[1]))));
    T k2 = fmaf_(T(Hr[2]), d0, fmaf_(T(Hr[4]), d1, fmaf_(T(Hr[5]), d2, T(L[2]))));
    Jet<T> V;
    V.v = fmaf_(T(0.5f), fmaf_(d0, T(L[0]) + k0, fmaf_(d1, T(L[1]) + k1, d2 * (T(L[2]) + k2))),
                T(M.P0[pop]) - MU.v);
    const T u0 = k0 - T(1);
    V.a = fmaf_(u0, MU.a, fmaf_(k1, SQ.a, k2 * TV.a));
    V.b = fmaf_(u0, MU.b, fmaf_(k1, SQ.b, k2 * TV.b));
    // H u_a and H u_b
    T wa0 = fmaf_(T(Hr[0]), MU.a, fmaf_(T(Hr[1]), SQ.a, T(Hr[2]) * TV.a));
    T wa1 = fmaf_(T(Hr[1]), MU.a, fmaf_(T(Hr[3]), SQ.a, T(Hr[4]) * TV.a));
    T wa2 = fmaf_(T(Hr[2]), MU.a, fmaf_(T(Hr[4]), SQ.a, T(Hr[5]) * TV.a));
    T wb0 = fmaf_(T(Hr[0]), MU.b, fmaf_(T(Hr[1]), SQ.b, T(Hr[2]) * TV.b));
    T wb1 = fmaf_(T(Hr[1]), MU.b, fmaf_(T(Hr[3]), SQ.b, T(Hr[4]) * TV.b));
    T wb2 = fmaf_(T(Hr[2]), MU.b, fmaf_(T(Hr[4]), SQ.b, T(Hr[5]) * TV.b));
    V.aa = fmaf_(u0, MU.aa, fmaf_(k1, SQ.aa, fmaf_(k2, TV.aa,
           fmaf_(wa0, MU.a, fmaf_(wa1, SQ.a, wa2 * TV.a)))));
    V.ab = fmaf_(u0, MU.ab, fmaf_(k1, SQ.ab, fmaf_(k2, TV.ab,
           fmaf_(wa0, MU.b, fmaf_(wa1, SQ.b, wa2 * TV.b)))));
    V.bb = fmaf_(u0, MU.bb, fmaf_(k1, SQ.bb, fmaf_(k2, TV.bb,
           fmaf_(wb0, MU.b, fmaf_(wb1, SQ.b, wb2 * TV.b)))));
    Jet<T> Z = jmul(V, Q);                            // (V_thre - mu_V)/(sqrt2 sigma_V)
    T ez, e;
    erfc_and_gauss(Z.v, ez, e);
    // F = erfc(Z) / (2 tau_V): the factor 1/2 rides on erfc's chain coefficients
    T g1 = T(-0.5f * 1.1283791670955126f) * e;
    Jet<T> GZ = jchain(Z, T(0.5f) * ez, g1, T(-2) * Z.v * g1);
    return jmul(GZ, ITV);
}

// Per-instance parameters.
template <class T> struct InstParams { T S, b_e, a_e; };

// Drift of one region's 8 states given its coupling input c (eq. 1-4).
template <int VAR, class T>
VADX_HD void drift(const KModel &M, const T X[8], T c, T be, T ae, T dX[8])
{
    const T E = X[0], I = X[1], Cee = X[2], Cei = X[3], Cii = X[4];
    T exc = E + c + T(M.w_noise) * X[7];
    T xe0 = maxf_(exc + T(M.cF[0][0]), T(M.x_floor));
    T xi0 = maxf_(I + T(M.cF[0][1]), T(M.x_floor));
    T xe1 = maxf_(exc + T(M.cF[1][0]), T(M.x_floor));
    T xi1 = maxf_(I + T(M.cF[1][1]), T(M.x_floor));
    T muVe, muVi;
    constexpr bool EQ = (VAR & kVarEq) != 0;
    const TFShared<T> g0 = tf_shared<EQ>(M, xe0, xi0);
    Jet<T> Fe = transfer<EQ>(M, 0, g0, X[5], muVe);
    Jet<T> Fi;
    if constexpr ((VAR & kVarSame) != 0) {
        (void)xe1;
        (void)xi1;
        Fi = transfer<EQ>(M, 1, g0, X[6], muVi);
    } else {
        const TFShared<T> g1 = tf_shared<EQ>(M, xe1, xi1);
        Fi = transfer<EQ>(M, 1, g1, X[6], muVi);
    }
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
// [0, rate_max] with mean nu), |C_ei| <= sqrt(C_ee C_ii). Returns true when a
// bound was hit. (Non-finite values are detected on the drift, before they
// reach the state.)
template <class S> VADX_HD S clampv(S x, S lo, S hi, bool &hit)
{
    S y = mind_(maxd_(x, lo), hi);
    hit = hit || (y != x);
    return y;
}
template <class S> VADX_HD bool project(const KModel &M, S X[8])
{
    bool hit = false;
    const S rm = S(M.rate_max);
    X[0] = clampv(X[0], S(0), rm, hit);
    X[1] = clampv(X[1], S(0), rm, hit);
    X[2] = clampv(X[2], S(0), X[0] * (rm - X[0]), hit);
    X[4] = clampv(X[4], S(0), X[1] * (rm - X[1]), hit);
    S cb = sqr(X[2] * X[4]);
    X[3] = clampv(X[3], -cb, cb, hit);
    return hit;
}

// Flags of one step: a bound of the projection was hit, the drift was not
// finite (every state enters the rate drifts, so their sum carries any NaN).
enum { kStepNonfinite = 1u, kStepClamp = 2u };

// One step of stochastic Heun (or Euler-Maruyama) for one region. The drift
// is evaluated in T (float); the state X and its increments are accumulated
// in S (double), so the rounding of the state does not build up over the
// run. gdw is the OU increment (sigma/tau_OU) sqrt(dt) z. Returns kStep* flags.
template <int VAR, class T, class S>
VADX_HD uint32_t step_region(const KModel &M, int integrator, S dt, S X[8], T c, T be, T ae, S gdw)
{
    T xf[8], f0[8], f1[8];
    S Xt[8];
    for (int q = 0; q < 8; ++q) xf[q] = T(X[q]);
    drift<VAR>(M, xf, c, be, ae, f0);
    if (integrator == 1) {
        const uint32_t nf = finite_(f0[0] + f0[1]) ? 0u : kStepNonfinite;
        for (int q = 0; q < 8; ++q) X[q] = X[q] + dt * S(f0[q]);
        X[7] = X[7] + gdw;
        return nf | (project(M, X) ? kStepClamp : 0u);
    }
    for (int q = 0; q < 8; ++q) Xt[q] = X[q] + dt * S(f0[q]);
    Xt[7] = Xt[7] + gdw;
    bool hit = project(M, Xt);
    for (int q = 0; q < 8; ++q) xf[q] = T(Xt[q]);
    drift<VAR>(M, xf, c, be, ae, f1);
    const uint32_t nf = finite_((f0[0] + f0[1]) + (f1[0] + f1[1])) ? 0u : kStepNonfinite;
    const S hdt = S(0.5) * dt;
    for (int q = 0; q < 8; ++q) X[q] = X[q] + hdt * S(f0[q] + f1[q]);
    X[7] = X[7] + gdw;
    hit = project(M, X) || hit;
    return nf | (hit ? kStepClamp : 0u);
}

} // namespace vadx
