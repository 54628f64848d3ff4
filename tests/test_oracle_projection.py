"""Pins of the oracle's admissible-state projection and of its Euler-Maruyama
branch.

Projection (applied after every stage): rates lie in [0, r]; a quantity
confined to [0, r] with mean nu has variance at most nu (r - nu) (the
Bhatia-Davis inequality), and a covariance is bounded by the geometric mean of
the two variances (Cauchy-Schwarz). The pins check the bounds on the output,
that real distributions on [0, r] are never moved, idempotence, and that the
flag is raised exactly when a value moved.

Euler-Maruyama (the paper's own integrator, Section 2.5): on the linear OU
equation (eq. 4) one step is the AR(1) map OU' = (1 - dt/tau) OU +
(sigma/tau) sqrt(dt) z; noise-free, the error halves with dt (order 1)
against a tight adaptive integration of the same drift.
"""
import numpy as np
import pytest
from scipy import integrate

from paper_2311_13337_amd import inputs

E, I, CEE, CEI, CII, WE, WI, OU = range(8)
FLAG_CLAMP = 2


def _random_prestates(rng, r, n):
    X = np.zeros((n, 8))
    X[:, E] = rng.uniform(-0.2 * r, 1.2 * r, n)
    X[:, I] = rng.uniform(-0.2 * r, 1.2 * r, n)
    X[:, CEE] = rng.uniform(-0.05, 0.35, n) * r * r
    X[:, CII] = rng.uniform(-0.05, 0.35, n) * r * r
    X[:, CEI] = rng.uniform(-0.3, 0.3, n) * r * r
    X[:, WE] = rng.normal(0, 50, n)
    X[:, WI] = rng.normal(0, 1, n)
    X[:, OU] = rng.normal(0, 1e-3, n)
    # some pre-states already admissible, some with exactly one bound violated
    X[: n // 4, E] = rng.uniform(0, r, n // 4)
    X[: n // 4, I] = rng.uniform(0, r, n // 4)
    return X


@pytest.mark.parametrize("r", [1.0, 0.5, 2.0])
def test_projection_output_satisfies_every_bound(oracle, r):
    m = oracle.model(rate_max=r)
    rng = np.random.default_rng(int(r * 10))
    for X in _random_prestates(rng, r, 3000):
        Y, fl = oracle.project(m, X)
        assert 0.0 <= Y[E] <= r and 0.0 <= Y[I] <= r
        assert 0.0 <= Y[CEE] <= Y[E] * (r - Y[E])
        assert 0.0 <= Y[CII] <= Y[I] * (r - Y[I])
        assert Y[CEI] ** 2 <= Y[CEE] * Y[CII] * (1 + 4e-16)
        # adaptation currents and noise are not projected
        assert np.array_equal(Y[[WE, WI, OU]], X[[WE, WI, OU]])


@pytest.mark.parametrize("r", [1.0, 0.5])
def test_projection_is_idempotent_and_flags_exactly_when_a_value_moved(oracle, r):
    m = oracle.model(rate_max=r)
    rng = np.random.default_rng(5)
    moved = 0
    for X in _random_prestates(rng, r, 3000):
        Y, fl = oracle.project(m, X)
        assert (fl == FLAG_CLAMP) == (not np.array_equal(X, Y)) and fl in (0, FLAG_CLAMP)
        moved += fl != 0
        Z, fl2 = oracle.project(m, Y)
        assert np.array_equal(Z, Y) and fl2 == 0
    assert 0 < moved < 3000


@pytest.mark.parametrize("r", [1.0, 0.25])
def test_moments_of_real_distributions_pass_unchanged(oracle, r):
    """Mean and covariance of any joint distribution of (nu_e, nu_i) on
    [0, r]^2 are admissible, so the projection leaves them bit-identical and
    raises no flag: the bounds never cut a state the moment equations could
    describe."""
    m = oracle.model(rate_max=r)
    rng = np.random.default_rng(17)
    for trial in range(2000):
        k = rng.integers(2, 12)
        pts = rng.uniform(0, r, (k, 2))
        if trial % 3 == 0:                       # mass near the edges
            pts = np.where(rng.random((k, 2)) < 0.5, rng.uniform(0, 0.02 * r, (k, 2)),
                           rng.uniform(0.98 * r, r, (k, 2)))
        p = rng.dirichlet(np.ones(k))
        mu = p @ pts
        d = pts - mu
        C = (d * p[:, None]).T @ d
        X = np.array([mu[0], mu[1], C[0, 0], C[0, 1], C[1, 1], 3.0, 0.0, 1e-4])
        # drop states within rounding of a bound: the theorems hold exactly
        # only in exact arithmetic
        if (C[0, 0] > mu[0] * (r - mu[0]) * (1 - 1e-12) or C[1, 1] > mu[1] * (r - mu[1]) * (1 - 1e-12)
                or C[0, 1] ** 2 > C[0, 0] * C[1, 1] * (1 - 1e-12)):
            continue
        Y, fl = oracle.project(m, X)
        assert fl == 0 and np.array_equal(X, Y)


def test_projection_bounds_are_sharp(oracle):
    """Each bound is attained by a distribution: a two-point law on {0, r}
    reaches nu (r - nu); perfectly correlated rates reach sqrt(C_ee C_ii).
    Beyond the bound, the projection lands on it."""
    r = 1.0
    m = oracle.model(rate_max=r)
    for p in (0.1, 0.37, 0.5, 0.8):
        nu = p * r
        bound = nu * (r - nu)
        Y, fl = oracle.project(m, [nu, nu, 1.5 * bound, 0.0, 3 * bound, 0, 0, 0])
        assert fl == FLAG_CLAMP and Y[CEE] == bound and Y[CII] == bound
        cee, cii = 0.3 * bound, 0.7 * bound
        Y, fl = oracle.project(m, [nu, nu, cee, -2.0, cii, 0, 0, 0])
        assert fl == FLAG_CLAMP and Y[CEI] == -np.sqrt(cee * cii)
    # negative rates and variances go to zero, and with them the covariance
    Y, fl = oracle.project(m, [-0.01, 0.3, -1e-4, 0.02, 0.05, 0, 0, 0])
    assert fl == FLAG_CLAMP and Y[E] == 0.0 and Y[CEE] == 0.0 and Y[CEI] == 0.0


def test_euler_on_linear_ou_is_exact_ar1(oracle):
    m = oracle.model()
    rng = np.random.default_rng(23)
    for dt in (0.05, 0.1, 0.2):
        a = 1 - dt / m.tau_OU
        s = (m.sigma_OU / m.tau_OU) * np.sqrt(dt)
        X = np.array([0.01, 0.01, 0, 0, 0, 0, 0, 0.0])
        for _ in range(50):
            X[OU] = rng.normal(0, 3e-4)
            z = rng.standard_normal()
            Y, _ = oracle.step_region(m, X, 0.0, 0.0, 0.0, z, dt, integrator=1)
            np.testing.assert_allclose(Y[OU], a * X[OU] + s * z, rtol=1e-13, atol=1e-22)


def test_euler_ou_stationary_statistics(oracle):
    """The Euler OU chain driven by the Philox normals of a whole run has the
    AR(1) stationary variance s^2 / (1 - a^2) and lag-1 autocorrelation a."""
    m = oracle.model()
    conn = inputs.synthetic_connectome(1, seed=3)
    b = inputs._batch([0.0], [0.0], [0.0], [4.0])
    n = 40000
    cfg = inputs.RunConfig(n_steps=n, n_trace_steps=n, seed=7, transient_steps=0)
    r = oracle.run(m, cfg, conn, b, integrator=1, want_fc=False, n_threads=1)
    x = r["trace"][0, 2000:, OU, 0]
    dt = cfg.dt_ms
    a = 1 - dt / m.tau_OU
    s = (m.sigma_OU / m.tau_OU) * np.sqrt(dt)
    var = s * s / (1 - a * a)
    # effective sample size of an AR(1) series for the variance and lag-1 estimates
    neff = len(x) * (1 - a * a) / (1 + a * a)
    assert abs(x.var() / var - 1) < 4 * np.sqrt(2 / neff)
    rho = np.corrcoef(x[:-1], x[1:])[0, 1]
    assert abs(rho - a) < 4 * np.sqrt((1 - a * a) / neff) + 4 * (1 - a * a) / np.sqrt(len(x))


def test_euler_is_first_order(oracle):
    """Noise-free single node away from any bound: halving dt halves the error
    against an adaptive integration of the oracle's own drift (drive
    0.3e-3 kHz: the trajectory stays inside the admissible set)."""
    m = oracle.model(cF_ee=0.3e-3, cF_ie=0.3e-3)
    X0 = np.array([0.006, 0.012, 1e-6, 1e-6, 2e-6, 3.0, 0, 0])
    be, ae, T = 30.0, 2.0, 20.0

    def euler(dt):
        X = X0.copy()
        for _ in range(int(round(T / dt))):
            X, fl = oracle.step_region(m, X, 0.0, be, ae, 0.0, dt, integrator=1)
            assert fl == 0
        return X
    sol = integrate.solve_ivp(lambda t, y: oracle.drift(m, y, 0.0, be, ae), (0.0, T), X0,
                              method="DOP853", rtol=1e-12, atol=1e-16)
    ref = sol.y[:, -1]
    e1 = np.abs(euler(0.2) - ref)[[E, I]].max()
    e2 = np.abs(euler(0.1) - ref)[[E, I]].max()
    assert 1.8 < e1 / e2 < 2.2
