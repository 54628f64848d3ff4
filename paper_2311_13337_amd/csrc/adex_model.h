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
// (xe, xi) enter eq. 1 only through the gradient and through the Hessian's
// contraction with the covariance matrix C of the inputs, q = tr(C H) / 2, so
// every quantity is carried as a 4-component jet (value, gradient, q): the
// product and chain rules hold for q with the bilinear term grad x . C grad y.
// The derivatives of every quantity that depends on the inputs only through G
// are formed from its scalar derivatives in G, and mu_V's from its closed form.
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
    float Hq[2][6];             // Hraw with the diagonal halved: sum Hq_kl M_kl over k <= l = sum_kl H_kl M_kl / 2
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

// A value with its gradient (a = d/dxe, b = d/dxi) and q = tr(C H) / 2, H its
// Hessian in (xe, xi), C the covariance matrix of (xe, xi).
template <class T> struct QJet { T v, a, b, q; };

// Covariance matrix C of the inputs (C_ee, C_ei, C_ii) and its products with
// n = (a_e, a_i), the gradient direction of G: (nx, ny) = C n, qG = n . C n / 2.
template <class T> struct Cov { T ee, ei, ii, nx, ny, qG; };

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
VADX_HD float maxd_(float a, float b) { return __builtin_fmaxf(a, b); }
VADX_HD float mind_(float a, float b) { return __builtin_fminf(a, b); }
VADX_HD bool finite_(float x) { return __builtin_isfinite(x); }
VADX_HD float fmaf_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
VADX_HD float absf_(float x) { return __builtin_fabsf(x); }
VADX_HD float selectf(bool c, float a, float b) { return c ? a : b; }
VADX_HD float maxf_(float a, float b) { return __builtin_fmaxf(a, b); }

// ---------------------------------------------------------------- jet algebra
// grad x . C grad y
template <class T> VADX_HD T cdot(const Cov<T> &C, T xa, T xb, T ya, T yb)
{
    return fmaf_(xa, fmaf_(C.ee, ya, C.ei * yb), xb * fmaf_(C.ei, ya, C.ii * yb));
}
// C grad x
template <class T> VADX_HD void cvec(const Cov<T> &C, T xa, T xb, T &cx, T &cy)
{
    cx = fmaf_(C.ee, xa, C.ei * xb);
    cy = fmaf_(C.ei, xa, C.ii * xb);
}
template <class T> VADX_HD QJet<T> qmul(const QJet<T> &x, const QJet<T> &y, const Cov<T> &C)
{
    QJet<T> r;
    r.v = x.v * y.v;
    r.a = fmaf_(x.a, y.v, x.v * y.a);
    r.b = fmaf_(x.b, y.v, x.v * y.b);
    r.q = fmaf_(x.q, y.v, fmaf_(x.v, y.q, cdot(C, x.a, x.b, y.a, y.b)));
    return r;
}
template <class T> VADX_HD QJet<T> qadd(const QJet<T> &x, const QJet<T> &y)
{
    return QJet<T>{x.v + y.v, x.a + y.a, x.b + y.b, x.q + y.q};
}
// f(x) given f, f', f'' at x.v: q = f' q_x + f'' (grad x . C grad x) / 2
template <class T> VADX_HD QJet<T> qchain(const QJet<T> &x, T f0, T f1, T f2, const Cov<T> &C)
{
    T cx, cy;
    cvec(C, x.a, x.b, cx, cy);
    const T half_quad = T(0.5f) * fmaf_(x.a, cx, x.b * cy);
    return QJet<T>{f0, f1 * x.a, f1 * x.b, fmaf_(f1, x.q, f2 * half_quad)};
}
// a function of G = g_L + aE xe + aI xi only: f, f', f'' in G
template <class T> VADX_HD QJet<T> qofG(T f0, T f1, T f2, T aE, T aI, const Cov<T> &C)
{
    return QJet<T>{f0, f1 * aE, f1 * aI, f2 * C.qG};
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

// The parts of the transfer function that depend on the inputs only through
// xe, xi, G = g_L + a_e xe + a_i xi and the input covariance, not on the
// population: shared by the two populations when their inputs coincide.
// EQ: tau_e == tau_i, so d_i = d_e, 1/tau_V = d_e and sigma_V^2 = (A_e + A_i) d_e / 2.
template <class T> struct TFShared {
    T xe, xi, r, r2, r3;
    T de, he1, he2;             // d_e = 1/(C_m/G + tau_e) and its first two derivatives in G
    T cexe, cixi;               // c_e xe, c_i xi
    T pq0;                      // the xe, xi terms of q(Pi): (C_ee c_i 2bI^2 xi + C_ii c_e 2bE^2 xe) / 2
    // tau_e == tau_i only: phi = d_e / G^4 and the G-derivative terms of
    // S2 = Pi phi; the jets of 1/tau_V = d_e and tau_V = C_m/G + tau_e and the
    // C-products of their gradients
    T phi, phi1aE, phi1aI, phi1nx, phi1ny, phi2qG;
    QJet<T> ITV, TV;
    T itv1nx, itv1ny, itv2qG;   // d_e' (C n), d_e'' qG
    T tv1nx, tv1ny, m22;        // tau_V' (C n), grad tau_V . C grad tau_V
};

template <bool EQ, class T>
VADX_HD TFShared<T> tf_shared(const KModel &M, T xe, T xi, const Cov<T> &C)
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
    g.pq0 = T(0.5f) * fmaf_(C.ee * T(M.ci2bI2), xi, C.ii * T(M.ce2bE2) * xe);
    if constexpr (EQ) {
        // (ln phi)' = -(3 + tau d_e)/G, phi'' = phi (12 + 6 tau d_e + 2 (tau d_e)^2) / G^2
        T td = T(M.tau_e) * g.de;
        g.phi = g.r2 * g.r2 * g.de;
        const T phi1 = -g.phi * g.r * (T(3) + td);
        const T phi2 = g.phi * g.r2 * fmaf_(td, fmaf_(T(2), td, T(6)), T(12));
        g.phi1aE = phi1 * aE;
        g.phi1aI = phi1 * aI;
        g.phi1nx = phi1 * C.nx;
        g.phi1ny = phi1 * C.ny;
        g.phi2qG = phi2 * C.qG;
        g.ITV = qofG(g.de, g.he1, g.he2, aE, aI, C);
        g.itv1nx = g.he1 * C.nx;
        g.itv1ny = g.he1 * C.ny;
        g.itv2qG = g.ITV.q;
        // tau_V = T_eff + tau_e = C_m/G + tau_e
        const T tv1 = -T(M.Cm) * g.r2;
        g.TV = qofG(fmaf_(T(M.Cm), g.r, T(M.tau_e)), tv1, T(2) * T(M.Cm) * g.r3, aE, aI, C);
        g.tv1nx = tv1 * C.nx;
        g.tv1ny = tv1 * C.ny;
        g.m22 = T(2) * tv1 * tv1 * C.qG;
    }
    return g;
}

// Transfer function of population `pop` with its gradient and q in (xe, xi).
// Also returns mu_V (value) for the adaptation equation.
template <bool EQ, class T>
VADX_HD QJet<T> transfer(const KModel &M, int pop, const TFShared<T> &g, const Cov<T> &C, T W,
                         T &muV_out)
{
    const T aE = T(M.aE), aI = T(M.aI);
    const T xe = g.xe, xi = g.xi, r = g.r, r2 = g.r2, r3 = g.r3;
    // mu_V through A = (E_e - mu_V) G = alpha_e + beta_e xi (linear in xi) and
    // B = (E_i - mu_V) G = alpha_i + beta_i xe (linear in xe): mu_V = E_e - A/G,
    // Hessian -2A/G^3 n n^T + (bE/G^2)(n e_i^T + e_i n^T), so
    // q = -2A/G^3 qG + bE/G^2 (C n)_i
    T c0 = T(M.gLEL[pop]) - W;
    T A = fmaf_(T(M.bE), xi, T(M.EegL) - c0);
    T B = fmaf_(T(M.bI), xe, T(M.EigL) - c0);
    T Ar2 = A * r2, Ar3 = T(2) * A * r3, bEr2 = T(M.bE) * r2;
    QJet<T> MU;
    MU.v = fmaf_(-A, r, T(M.Ee));
    MU.a = Ar2 * aE;
    MU.b = fmaf_(Ar2, aI, -T(M.bE) * r);
    MU.q = fmaf_(bEr2, C.ny, -Ar3 * C.qG);
    muV_out = MU.v;
    // shot-noise weights A_s = K_s x_s (tau_s U_s)^2 with U_e = Q_e A/G^2,
    // U_i = Q_i B/G^2: A_e + A_i = Pi / G^4 with the cubic
    // Pi = c_e xe A^2 + c_i xi B^2 (c_s = K_s tau_s^2 Q_s^2), whose derivatives
    // are exact polynomials
    const T ce = T(M.ce), ci = T(M.ci);
    const T cexe = g.cexe, cixi = g.cixi;
    T A2 = A * A, B2 = B * B;
    QJet<T> S2, ITV, TV;                             // 2 sigma_V^2, 1/tau_V, tau_V
    if constexpr (EQ) {
        QJet<T> PI;
        PI.v = fmaf_(cexe, A2, cixi * B2);
        PI.a = fmaf_(ce, A2, T(M.ci2bI) * xi * B);
        PI.b = fmaf_(T(M.ce2bE) * xe, A, ci * B2);
        PI.q = fmaf_(C.ei, fmaf_(T(M.ce2bE), A, T(M.ci2bI) * B), g.pq0);
        // S2 = Pi phi(G)
        S2.v = PI.v * g.phi;
        S2.a = fmaf_(PI.a, g.phi, PI.v * g.phi1aE);
        S2.b = fmaf_(PI.b, g.phi, PI.v * g.phi1aI);
        S2.q = fmaf_(PI.q, g.phi, fmaf_(PI.v, g.phi2qG, fmaf_(PI.a, g.phi1nx, PI.b * g.phi1ny)));
        ITV = g.ITV;
        TV = g.TV;
    } else {
        // A_e = c_e xe A^2 / G^4 and A_i = c_i xi B^2 / G^4 weighted separately
        QJet<T> Ae, Ai;
        Ae.v = cexe * A2; Ae.a = ce * A2; Ae.b = T(M.ce2bE) * xe * A;
        Ae.q = fmaf_(C.ei * T(M.ce2bE), A, T(0.5f) * C.ii * T(M.ce2bE2) * xe);
        Ai.v = cixi * B2; Ai.a = T(M.ci2bI) * xi * B; Ai.b = ci * B2;
        Ai.q = fmaf_(C.ei * T(M.ci2bI), B, T(0.5f) * C.ee * T(M.ci2bI2) * xi);
        T r4 = r2 * r2;
        QJet<T> R4 = qofG(r4, T(-4) * r4 * r, T(20) * r4 * r2, aE, aI, C);
        Ae = qmul(Ae, R4, C);
        Ai = qmul(Ai, R4, C);
        QJet<T> De = qofG(g.de, g.he1, g.he2, aE, aI, C);
        T di = rcp(fmaf_(T(M.Cm), r, T(M.tau_i)));
        T qi = di * r;
        T hi1 = T(M.Cm) * qi * qi;
        const T hi2 = T(-2) * T(M.tau_i) * hi1 * qi;
        QJet<T> Di = qofG(di, hi1, hi2, aE, aI, C);
        S2 = qadd(qmul(Ae, De, C), qmul(Ai, Di, C));
        // 1/tau_V = (A_e d_e + A_i d_i)/(A_e + A_i) = d_e + w (d_i - d_e) with
        // w = A_i/(A_e + A_i): a weighted mean of d_e, d_i whose derivatives do
        // not cancel when one source dominates (the ratio form loses them in FP32).
        QJet<T> As = qadd(Ae, Ai);
        T ra = rcp(As.v);
        T ra2 = ra * ra;
        QJet<T> RA = qchain(As, ra, -ra2, T(2) * ra2 * ra, C);
        QJet<T> Wi = qmul(Ai, RA, C);
        QJet<T> Dd = qofG(di - g.de, hi1 - g.he1, hi2 - g.he2, aE, aI, C);
        ITV = qadd(De, qmul(Wi, Dd, C));
        T itv = rcp(ITV.v);
        T itv2 = itv * itv;
        TV = qchain(ITV, itv, -itv2, T(2) * itv2 * itv, C);
    }
    // q = S2^(-1/2) = 1/(sqrt2 sigma_V);  (x^-1/2)' = -q^3/2, '' = 3 q^5/4
    // SQ = sqrt(S2) = sqrt2 sigma_V;      (x^1/2)' = q/2,     '' = -q^3/4
    T cs2x, cs2y;
    cvec(C, S2.a, S2.b, cs2x, cs2y);                 // C grad S2
    const T hq2 = T(0.5f) * fmaf_(S2.a, cs2x, S2.b * cs2y);
    T q = rsq(S2.v);
    T q2 = q * q, q3 = q2 * q;
    const T f1 = T(-0.5f) * q3, h1 = T(0.5f) * q;
    QJet<T> Q{q, f1 * S2.a, f1 * S2.b, fmaf_(f1, S2.q, T(0.75f) * q3 * q2 * hq2)};
    QJet<T> SQ{S2.v * q, h1 * S2.a, h1 * S2.b, fmaf_(h1, S2.q, T(-0.25f) * q3 * hq2)};
    // V = V_thre - mu_V with the threshold polynomial p of Table 1 written in
    // the offsets d = u - c of u = (mu_V, SQ, tau_V) from the centre c of its
    // normalisation: p = P0 + L.d + d.H d / 2 with L_k = P_k s_k and the constant
    // Hessian H_kl = s_k s_l d2p/dn_k dn_l, so grad p = L + H d, and
    // q(V) = sum_k (dV/du_k) q(u_k) + sum_kl H_kl (grad u_k . C grad u_l) / 2.
    const float *L = M.plin[pop], *Hr = M.Hraw[pop], *Hq = M.Hq[pop];
    T d0 = MU.v - T(M.pc[0]), d1 = SQ.v - T(M.pc[1]), d2 = TV.v - T(M.pc[2]);
    T k0 = fmaf_(T(Hr[0]), d0, fmaf_(T(Hr[1]), d1, fmaf_(T(Hr[2]), d2, T(L[0]))));
    T k1 = fmaf_(T(Hr[1]), d0, fmaf_(T(Hr[3]), d1, fmaf_(T(Hr[4]), d2, T(L[1]))));
    T k2 = fmaf_(T(Hr[2]), d0, fmaf_(T(Hr[4]), d1, fmaf_(T(Hr[5]), d2, T(L[2]))));
    QJet<T> V;
    V.v = fmaf_(T(0.5f), fmaf_(d0, T(L[0]) + k0, fmaf_(d1, T(L[1]) + k1, d2 * (T(L[2]) + k2))),
                T(M.P0[pop]) - MU.v);
    const T u0 = k0 - T(1);
    V.a = fmaf_(u0, MU.a, fmaf_(k1, SQ.a, k2 * TV.a));
    V.b = fmaf_(u0, MU.b, fmaf_(k1, SQ.b, k2 * TV.b));
    // M_kl = grad u_k . C grad u_l with C grad SQ = (q/2) C grad S2 and
    // C grad tau_V = tau_V' C n in the tau_e == tau_i case
    T cm0x, cm0y, ct2x, ct2y, m22;
    cvec(C, MU.a, MU.b, cm0x, cm0y);
    if constexpr (EQ) {
        ct2x = g.tv1nx;
        ct2y = g.tv1ny;
        m22 = g.m22;
    } else {
        cvec(C, TV.a, TV.b, ct2x, ct2y);
        m22 = fmaf_(TV.a, ct2x, TV.b * ct2y);
    }
    const T c1x = h1 * cs2x, c1y = h1 * cs2y;
    const T m00 = fmaf_(MU.a, cm0x, MU.b * cm0y);
    const T m01 = fmaf_(MU.a, c1x, MU.b * c1y);
    const T m02 = fmaf_(MU.a, ct2x, MU.b * ct2y);
    const T m11 = h1 * h1 * T(2) * hq2;
    const T m12 = fmaf_(SQ.a, ct2x, SQ.b * ct2y);
    V.q = fmaf_(u0, MU.q, fmaf_(k1, SQ.q, fmaf_(k2, TV.q,
          fmaf_(T(Hq[0]), m00, fmaf_(T(Hq[3]), m11, fmaf_(T(Hq[5]), m22,
          fmaf_(T(Hq[1]), m01, fmaf_(T(Hq[2]), m02, T(Hq[4]) * m12))))))));
    // Z = V q: (V_thre - mu_V)/(sqrt2 sigma_V); C grad q = f1 C grad S2
    QJet<T> Z;
    Z.v = V.v * Q.v;
    Z.a = fmaf_(V.a, Q.v, V.v * Q.a);
    Z.b = fmaf_(V.b, Q.v, V.v * Q.b);
    Z.q = fmaf_(V.q, Q.v, fmaf_(V.v, Q.q, f1 * fmaf_(V.a, cs2x, V.b * cs2y)));
    T ez, e;
    erfc_and_gauss(Z.v, ez, e);
    // F = erfc(Z) / (2 tau_V): the factor 1/2 rides on erfc's chain coefficients
    T g1 = T(-0.5f * 1.1283791670955126f) * e;
    QJet<T> GZ = qchain(Z, T(0.5f) * ez, g1, T(-2) * Z.v * g1, C);
    if constexpr (EQ) {
        // F = GZ (1/tau_V) with 1/tau_V = d_e(G)
        QJet<T> F;
        F.v = GZ.v * ITV.v;
        F.a = fmaf_(GZ.a, ITV.v, GZ.v * ITV.a);
        F.b = fmaf_(GZ.b, ITV.v, GZ.v * ITV.b);
        F.q = fmaf_(GZ.q, ITV.v, fmaf_(GZ.v, g.itv2qG, fmaf_(GZ.a, g.itv1nx, GZ.b * g.itv1ny)));
        return F;
    } else {
        return qmul(GZ, ITV, C);
    }
}

// Parameters of one instance (the axes of a sweep, Table 4): spike-frequency
// and subthreshold adaptation b_e, a_e, noise weight, 1/tau_w of the
// excitatory population and the external drives c_F (population, input).
template <class T> struct InstModel {
    T be, ae, w_noise, inv_tauw_e;
    T cF[2][2];
};

// The instance parameters equal to the model's, with b_e and a_e given.
template <class T> VADX_HD InstModel<T> inst_model(const KModel &M, T be, T ae)
{
    InstModel<T> P;
    P.be = be;
    P.ae = ae;
    P.w_noise = T(M.w_noise);
    P.inv_tauw_e = T(M.inv_tauw[0]);
    P.cF[0][0] = T(M.cF[0][0]);
    P.cF[0][1] = T(M.cF[0][1]);
    P.cF[1][0] = T(M.cF[1][0]);
    P.cF[1][1] = T(M.cF[1][1]);
    return P;
}

// Drift of one region's 8 states given its coupling input c (eq. 1-4).
// VAR & kVarSame requires P.cF[0] == P.cF[1] (both populations see the same inputs).
template <int VAR, class T>
VADX_HD void drift(const KModel &M, const T X[8], T c, const InstModel<T> &P, T dX[8])
{
    const T E = X[0], I = X[1], Cee = X[2], Cei = X[3], Cii = X[4];
    const T be = P.be, ae = P.ae;
    T exc = E + c + P.w_noise * X[7];
    T xe0 = maxf_(exc + P.cF[0][0], T(M.x_floor));
    T xi0 = maxf_(I + P.cF[0][1], T(M.x_floor));
    T xe1 = maxf_(exc + P.cF[1][0], T(M.x_floor));
    T xi1 = maxf_(I + P.cF[1][1], T(M.x_floor));
    // the covariance of the inputs (xe, xi) is that of the rates (E, I)
    Cov<T> C;
    C.ee = Cee;
    C.ei = Cei;
    C.ii = Cii;
    cvec(C, T(M.aE), T(M.aI), C.nx, C.ny);
    C.qG = T(0.5f) * fmaf_(T(M.aE), C.nx, T(M.aI) * C.ny);
    T muVe, muVi;
    constexpr bool EQ = (VAR & kVarEq) != 0;
    const TFShared<T> g0 = tf_shared<EQ>(M, xe0, xi0, C);
    QJet<T> Fe = transfer<EQ>(M, 0, g0, C, X[5], muVe);
    QJet<T> Fi;
    if constexpr ((VAR & kVarSame) != 0) {
        (void)xe1;
        (void)xi1;
        Fi = transfer<EQ>(M, 1, g0, C, X[6], muVi);
    } else {
        const TFShared<T> g1 = tf_shared<EQ>(M, xe1, xi1, C);
        Fi = transfer<EQ>(M, 1, g1, C, X[6], muVi);
    }
    const T iT = T(M.invT);
    T fe = Fe.v - E, fi = Fi.v - I;
    // eq. 1: T dnu/dt = (F - nu) + 1/2 C_ee F_ee + C_ei F_ei + 1/2 C_ii F_ii = (F - nu) + q(F)
    dX[0] = iT * (Fe.q + fe);
    dX[1] = iT * (Fi.q + fi);
    // eq. 2
    dX[2] = iT * fmaf_(Fe.v * (iT - Fe.v), T(M.invNe),
                       fmaf_(fe, fe, T(2) * (fmaf_(Cee, Fe.a, Cei * Fe.b) - Cee)));
    dX[3] = iT * fmaf_(fe, fi, fmaf_(Cee, Fi.a, fmaf_(Cei, Fi.b + Fe.a,
                                                        fmaf_(Cii, Fe.b, T(-2) * Cei))));
    dX[4] = iT * fmaf_(Fi.v * (iT - Fi.v), T(M.invNi),
                       fmaf_(fi, fi, T(2) * (fmaf_(Cii, Fi.b, Cei * Fi.a) - Cii)));
    // eq. 3 (AdEx form, subthreshold term over tau_w)
    dX[5] = fmaf_(be, E, P.inv_tauw_e * fmaf_(ae, muVe - T(M.EL[0]), -X[5]));
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
// Below C_ei^2 < C_ee C_ii * proj_skip (each side rounded) |C_ei| is below
// sqrt(C_ee C_ii) in any rounding: 1 - 2^-40 in double, 1 - 1e-5 in single
// precision (margins of many ulps over the products' and the root's rounding).
VADX_HD double proj_skip(double) { return 0.99999999999909051; }
VADX_HD float proj_skip(float) { return 0.99999f; }
template <class S> VADX_HD bool project(const KModel &M, S X[8])
{
    bool hit = false;
    const S rm = S(M.rate_max);
    X[0] = clampv(X[0], S(0), rm, hit);
    X[1] = clampv(X[1], S(0), rm, hit);
    X[2] = clampv(X[2], S(0), X[0] * (rm - X[0]), hit);
    X[4] = clampv(X[4], S(0), X[1] * (rm - X[1]), hit);
    // |C_ei| <= sqrt(C_ee C_ii): the square root is taken only where the bound
    // may bind. Below C_ei^2 < C_ee C_ii (1 - 2^-40) (each side rounded),
    // |C_ei| < sqrt(C_ee C_ii) in any rounding, so the clamp would leave C_ei
    // unchanged and flag nothing.
    const S p = X[2] * X[4];
    if (X[3] * X[3] >= p * proj_skip(S(0))) {
        S cb = sqr(p);
        X[3] = clampv(X[3], -cb, cb, hit);
    }
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
VADX_HD uint32_t step_region(const KModel &M, int integrator, S dt, S X[8], T c,
                             const InstModel<T> &P, S gdw)
{
    T xf[8], f0[8], f1[8];
    for (int q = 0; q < 8; ++q) xf[q] = T(X[q]);
    drift<VAR>(M, xf, c, P, f0);
    if (integrator == 1) {
        const uint32_t nf = finite_(f0[0] + f0[1]) ? 0u : kStepNonfinite;
        for (int q = 0; q < 8; ++q) X[q] = X[q] + dt * S(f0[q]);
        X[7] = X[7] + gdw;
        return nf | (project(M, X) ? kStepClamp : 0u);
    }
    // predictor in single precision: it feeds only the second drift, which
    // takes single-precision inputs anyway
    for (int q = 0; q < 8; ++q) xf[q] = fmaf_(T(dt), f0[q], xf[q]);
    xf[7] = xf[7] + T(gdw);
    bool hit = project(M, xf);
    drift<VAR>(M, xf, c, P, f1);
    const uint32_t nf = finite_((f0[0] + f0[1]) + (f1[0] + f1[1])) ? 0u : kStepNonfinite;
    const S hdt = S(0.5) * dt;
    for (int q = 0; q < 8; ++q) X[q] = X[q] + hdt * S(f0[q] + f1[q]);
    X[7] = X[7] + gdw;
    hit = project(M, X) || hit;
    return nf | (hit ? kStepClamp : 0u);
}

} // namespace vadx
