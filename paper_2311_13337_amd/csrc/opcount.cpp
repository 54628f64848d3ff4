// opcount.cpp -- exact arithmetic count of one region-step of the integration
// kernel, obtained by running the same templated model code (adex_model.h) on
// the host with a scalar type that counts its operations. Used for roofline
// accounting: add/sub/mul/compare-free min-max = 1 FLOP, fused multiply-add =
// 2 FLOPs, each transcendental (reciprocal, (reciprocal) square root, exp2,
// log2) = 1 FLOP and also tallied on its own.
#include <cmath>
#include <cstdint>

#include "vadx.h"

namespace vadx {
struct OpTally {
    double flop32 = 0, flop64 = 0, trans32 = 0, trans64 = 0;
};
static thread_local OpTally g_tally;

template <class U> struct Cnt {
    U v;
    Cnt() : v(0) {}
    Cnt(double x) : v((U)x) {}
    template <class V> explicit Cnt(const Cnt<V> &o) : v((U)o.v) {}
    static void flop(double n) { (sizeof(U) == 8 ? g_tally.flop64 : g_tally.flop32) += n; }
    static void trans() { (sizeof(U) == 8 ? g_tally.trans64 : g_tally.trans32) += 1; flop(1); }
};
template <class U> Cnt<U> mk(U x) { Cnt<U> r; r.v = x; return r; }
template <class U> Cnt<U> operator+(Cnt<U> a, Cnt<U> b) { Cnt<U>::flop(1); return mk<U>(a.v + b.v); }
template <class U> Cnt<U> operator-(Cnt<U> a, Cnt<U> b) { Cnt<U>::flop(1); return mk<U>(a.v - b.v); }
template <class U> Cnt<U> operator*(Cnt<U> a, Cnt<U> b) { Cnt<U>::flop(1); return mk<U>(a.v * b.v); }
template <class U> Cnt<U> operator-(Cnt<U> a) { return mk<U>(-a.v); }
template <class U> bool operator<(Cnt<U> a, Cnt<U> b) { return a.v < b.v; }
template <class U> bool operator>(Cnt<U> a, Cnt<U> b) { return a.v > b.v; }
template <class U> bool operator>=(Cnt<U> a, Cnt<U> b) { return a.v >= b.v; }

using CF = Cnt<float>;
using CD = Cnt<double>;
inline CF rcp(CF x) { CF::trans(); return mk<float>(1.0f / x.v); }
inline CF rsq(CF x) { CF::trans(); return mk<float>(1.0f / std::sqrt(x.v)); }
inline CF sqr(CF x) { CF::trans(); return mk<float>(std::sqrt(x.v)); }
inline CD sqr(CD x) { CD::trans(); return mk<double>(std::sqrt(x.v)); }
inline CF ex2(CF x) { CF::trans(); return mk<float>(std::exp2(x.v)); }
inline CF lg2(CF x) { CF::trans(); return mk<float>(std::log2(x.v)); }
inline CF fmaf_(CF a, CF b, CF c) { CF::flop(2); return mk<float>(std::fma(a.v, b.v, c.v)); }
inline CF absf_(CF x) { return mk<float>(std::fabs(x.v)); }
inline CF selectf(bool c, CF a, CF b) { return c ? a : b; }
inline CF maxf_(CF a, CF b) { CF::flop(1); return mk<float>(std::fmax(a.v, b.v)); }
inline CD maxd_(CD a, CD b) { CD::flop(1); return mk<double>(std::fmax(a.v, b.v)); }
inline CD mind_(CD a, CD b) { CD::flop(1); return mk<double>(std::fmin(a.v, b.v)); }
inline CF maxd_(CF a, CF b) { CF::flop(1); return mk<float>(std::fmax(a.v, b.v)); }
inline CF mind_(CF a, CF b) { CF::flop(1); return mk<float>(std::fmin(a.v, b.v)); }
inline CD proj_skip(CD) { return CD(0.99999999999909051); }
inline CF proj_skip(CF) { return CF(0.99999); }
inline bool finite_(CF x) { return std::isfinite(x.v); }
template <class U> bool operator!=(Cnt<U> a, Cnt<U> b) { return a.v != b.v; }
} // namespace vadx

#include "adex_model.h"

#include "kmodel.h"

extern "C" vadx_status vadx_region_step_ops(int32_t integrator, double *flop32, double *flop64,
                                            double *transcendental)
{
    using namespace vadx;
    if (!flop32 || !flop64 || !transcendental || (integrator != 0 && integrator != 1))
        return VADX_E_ARG;
    g_tally = OpTally{};
    vadx_model mm;
    vadx_model_defaults(VADX_PRESET_LITERATURE_B, &mm);
    KModel M = make_kmodel(mm);
    CD X[8] = {CD(0.004), CD(0.01), CD(2e-6), CD(4e-6), CD(1e-5), CD(20.0), CD(0.0), CD(1e-4)};
    const CD dt(0.1), gdw(1e-5);
    const CF c(1e-3f), be(30.f), ae(2.f);
    const InstModel<CF> P = inst_model<CF>(M, be, ae);
    switch (model_variant(M)) {
    case 0: step_region<0, CF, CD>(M, integrator, dt, X, c, P, gdw); break;
    case 1: step_region<1, CF, CD>(M, integrator, dt, X, c, P, gdw); break;
    case 2: step_region<2, CF, CD>(M, integrator, dt, X, c, P, gdw); break;
    default: step_region<3, CF, CD>(M, integrator, dt, X, c, P, gdw); break;
    }
    // per-step extras of the kernel: coupling scale S*c, OU increment gdw*z, the
    // running time average, and one quarter of a Box-Muller pair evaluation
    // (two normals per pair: log, sqrt, sin, cos and 8 products/sums).
    g_tally.flop32 += 1 + 1 + 0.25 * (8 + 4);
    g_tally.flop64 += 1;
    g_tally.trans32 += 0.25 * 4;
    *flop32 = g_tally.flop32;
    *flop64 = g_tally.flop64;
    *transcendental = g_tally.trans32 + g_tally.trans64;
    return VADX_OK;
}
