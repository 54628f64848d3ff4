"""Pins of the oracle's transfer function (Section 2.2, Table 1) against things
other than itself: the printed Table 1, the membrane current balance solved as
an ODE, Campbell's theorem for the shot-noise membrane potential evaluated by
quadrature, the normal law from scipy, and numerical differentiation."""
import os

import numpy as np
import pytest
from scipy import integrate, stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_threshold_polynomial.txt")

# Operating points (xe, xi [kHz], W [pA]) spanning low/high rates and adaptation.
POINTS = [(0.0043, 0.004, 0.0), (0.001, 0.003, 10.0), (0.01, 0.02, 50.0), (0.02, 0.01, 0.0),
          (0.0008, 0.0001, 0.0), (0.05, 0.05, 200.0), (0.004, 0.012, 5.0), (0.1, 0.2, 1000.0),
          (0.0025, 0.009, 30.0), (0.03, 0.001, 0.0), (0.006, 0.015, 80.0), (0.2, 0.19, 3000.0)]


def _golden():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, *vals = line.split()
        rows[name] = np.array([float(v) for v in vals])
    return rows


def _norm_coords(m, muV, sV, tV):
    return ((muV - m.muV0) / m.dmuV0, (sV - m.sV0) / m.dsV0, (tV * m.g_L / m.C_m - m.tN0) / m.dtN0)


@pytest.mark.parametrize("pop,row", [(0, "RS"), (1, "FS")])
def test_threshold_polynomial_recovers_table1(oracle, pop, row):
    """Least-squares fit of the oracle's V_thre over the 10 monomials of Table 1
    recovers the printed coefficients in the printed column order."""
    m = oracle.model("paper-T1")
    A, y = [], []
    rng = np.random.default_rng(1)
    for _ in range(40):
        xe, xi, W = rng.uniform(0.0005, 0.08), rng.uniform(0.0005, 0.08), rng.uniform(0, 300)
        o = oracle.tf(m, pop, xe, xi, W)
        mm, ss, tt = _norm_coords(m, o[6], o[7], o[8])
        A.append([1, mm, ss, tt, mm * mm, ss * ss, tt * tt, mm * ss, mm * tt, ss * tt])
        y.append(o[9])
    coef = np.linalg.lstsq(np.array(A), np.array(y), rcond=None)[0]
    np.testing.assert_allclose(coef, _golden()[row], rtol=0, atol=1e-8)


def test_literature_preset_differs_from_table1_in_three_readings(oracle):
    g = _golden()
    lb = oracle.model("literature-B")
    dRS = np.nonzero(np.array(lb.P_e) != g["RS"])[0].tolist()
    dFS = np.nonzero(np.array(lb.P_i) != g["FS"])[0].tolist()
    assert dRS == [0, 9] and dFS == [1, 9]
    assert lb.P_e[9] == -g["RS"][9] and lb.P_i[9] == -g["FS"][9]


@pytest.mark.parametrize("pop", [0, 1])
@pytest.mark.parametrize("pt", POINTS[:6])
def test_muV_is_membrane_steady_state(oracle, pop, pt):
    """mu_V is where the conductance-based membrane equation
    C dV/dt = gL(EL-V) + ge(Ee-V) + gi(Ei-V) - W comes to rest."""
    m = oracle.model()
    xe, xi, W = pt
    o = oracle.tf(m, pop, xe, xi, W)
    ge = m.Q_e * m.tau_e * m.K_e * xe
    gi = m.Q_i * m.tau_i * m.K_i * xi
    EL = m.E_L_e if pop == 0 else m.E_L_i

    def rhs(t, V):
        return (m.g_L * (EL - V) + ge * (m.E_e - V) + gi * (m.E_i - V) - W) / m.C_m

    sol = integrate.solve_ivp(rhs, (0, 400 * m.C_m / m.g_L), [EL], rtol=1e-12, atol=1e-12)
    assert abs(sol.y[0, -1] - o[6]) < 1e-8


def _psp(m, src, muV, muG):
    """PSP of one synaptic event: exponential conductance Q exp(-t/tau) at
    driving force (E_s - muV) on a membrane of time constant C/muG."""
    Q, tau, Es = (m.Q_e, m.tau_e, m.E_e) if src == 0 else (m.Q_i, m.tau_i, m.E_i)
    Teff = m.C_m / muG
    U = Q * (Es - muV) / muG
    # U tau/(Teff - tau) (exp(-t/Teff) - exp(-t/tau)), written without the
    # cancellation at Teff ~ tau.
    slow, fast = max(Teff, tau), min(Teff, tau)
    delta = 1.0 / fast - 1.0 / slow

    def h(t):
        g = t if delta < 1e-13 else -np.expm1(-t * delta) / delta
        return U * tau * np.exp(-t / slow) * g / (slow * fast)
    return h, 80.0 * slow


@pytest.mark.parametrize("pt", POINTS)
def test_sigmaV_tauV_from_campbell_quadrature(oracle, pt):
    """sigma_V^2 = sum_s rate_s * int h_s^2 (Campbell) and tau_V = int of the
    autocovariance over the variance, with rate_s = K_s x_s."""
    m = oracle.model()
    xe, xi, W = pt
    o = oracle.tf(m, 0, xe, xi, W)
    muG = m.g_L + m.Q_e * m.tau_e * m.K_e * xe + m.Q_i * m.tau_i * m.K_i * xi
    var, acov_int = 0.0, 0.0
    for src, rate in ((0, m.K_e * xe), (1, m.K_i * xi)):
        h, tmax = _psp(m, src, o[6], muG)
        var += rate * integrate.quad(lambda t: h(t) ** 2, 0, tmax, limit=400, epsabs=0,
                                     epsrel=1e-12)[0]
        acov_int += rate * integrate.quad(h, 0, tmax, limit=400, epsabs=0,
                                          epsrel=1e-12)[0] ** 2 / 2.0
    np.testing.assert_allclose(o[7] ** 2, var, rtol=1e-8)
    np.testing.assert_allclose(o[8], acov_int / var, rtol=1e-8)


@pytest.mark.parametrize("pop", [0, 1])
@pytest.mark.parametrize("pt", POINTS)
def test_rate_is_normal_tail_over_tauV(oracle, pop, pt):
    """F tau_V = P(V > V_thre) with V ~ N(mu_V, sigma_V^2)."""
    m = oracle.model()
    o = oracle.tf(m, pop, *pt)
    expect = stats.norm.sf(o[9], loc=o[6], scale=o[7]) / o[8]
    np.testing.assert_allclose(o[0], expect, rtol=1e-10, atol=1e-300)


def test_single_source_closed_forms(oracle):
    """With only excitatory input the autocorrelation time is tau_eff + tau_e;
    at V_thre = mu_V the rate is 1 / (2 tau_V)."""
    m = oracle.model()
    xe = 0.004
    o = oracle.tf(m, 0, xe, 1e-300, 0.0)
    muG = m.g_L + m.Q_e * m.tau_e * m.K_e * xe
    np.testing.assert_allclose(o[8], m.C_m / muG + m.tau_e, rtol=1e-12)
    # Pick W so that mu_V equals V_thre: V_thre depends on W only through mu_V,
    # so solve the scalar equation by bisection on W.
    from scipy.optimize import brentq
    f = lambda W: oracle.tf(m, 0, 0.004, 0.004, W)[9] - oracle.tf(m, 0, 0.004, 0.004, W)[6]
    W0 = brentq(f, -500, 500, xtol=1e-14)
    o = oracle.tf(m, 0, 0.004, 0.004, W0)
    np.testing.assert_allclose(o[0], 1.0 / (2 * o[8]), rtol=1e-9)


def _richardson(f, x, h, order):
    def d(hh):
        if order == 1:
            return (f(x + hh) - f(x - hh)) / (2 * hh)
        return (f(x + hh) - 2 * f(x) + f(x - hh)) / (hh * hh)
    return (4 * d(h / 2) - d(h)) / 3


@pytest.mark.parametrize("pop", [0, 1])
@pytest.mark.parametrize("pt", POINTS[:10])
def test_jet_derivatives_match_numerical_differentiation(oracle, pop, pt):
    m = oracle.model()
    xe, xi, W = pt
    o = oracle.tf(m, pop, xe, xi, W)
    F = lambda a, b: oracle.tf(m, pop, a, b, W)[0]
    he, hi = 1e-3 * xe, 1e-3 * xi
    scale1 = abs(o[0]) / min(xe, xi) + 1e-300
    scale2 = abs(o[0]) / min(xe, xi) ** 2 + 1e-300
    d_e = _richardson(lambda a: F(a, xi), xe, he, 1)
    d_i = _richardson(lambda b: F(xe, b), xi, hi, 1)
    d_ee = _richardson(lambda a: F(a, xi), xe, he, 2)
    d_ii = _richardson(lambda b: F(xe, b), xi, hi, 2)
    d_ei = _richardson(lambda a: _richardson(lambda b: F(a, b), xi, hi, 1), xe, he, 1)
    assert abs(d_e - o[1]) <= 1e-6 * max(abs(o[1]), scale1)
    assert abs(d_i - o[2]) <= 1e-6 * max(abs(o[2]), scale1)
    assert abs(d_ee - o[3]) <= 1e-4 * max(abs(o[3]), scale2)
    assert abs(d_ei - o[4]) <= 1e-4 * max(abs(o[4]), scale2)
    assert abs(d_ii - o[5]) <= 1e-4 * max(abs(o[5]), scale2)
