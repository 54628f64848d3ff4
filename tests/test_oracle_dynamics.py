"""Pins of the oracle's moment equations (Section 2.1 eq. 1-4), stepper,
coupling (Section 2.2 eq. 5), time averaging (Section 2.4) and FC (eq. 6):
Gauss-Hermite expectations, scipy's Lyapunov solver, the binomial variance,
closed forms of linear recursions, brute force on tiny networks, numpy's
corrcoef and fixed points found with scipy."""
import numpy as np
import pytest
from scipy import linalg, optimize, stats

from paper_2311_13337_amd import inputs

E, I, CEE, CEI, CII, WE, WI, OU = range(8)


def _quad_model(oracle, rng, N_big=False):
    m = oracle.model()
    m.tf_kind = 1
    for p in range(2):
        m.q_F0[p] = rng.uniform(0.002, 0.02)
        m.q_g[p][0], m.q_g[p][1] = rng.uniform(-2, 2, 2)
        m.q_H[p][0], m.q_H[p][1], m.q_H[p][2] = rng.uniform(-300, 300, 3)
    m.cF_ee = m.cF_ei = m.cF_ie = m.cF_ii = 0.0
    m.w_noise = 0.0
    if N_big:
        m.N_e = m.N_i = 1e300
    return m


def _qF(m, p, x):
    g, H = m.q_g[p], m.q_H[p]
    return (m.q_F0[p] + g[0] * x[0] + g[1] * x[1]
            + 0.5 * H[0] * x[0] ** 2 + H[1] * x[0] * x[1] + 0.5 * H[2] * x[1] ** 2)


@pytest.mark.parametrize("seed", range(5))
def test_rate_equation_is_expected_F_over_gaussian_rates(oracle, seed):
    """Eq. (1): for a quadratic F, F + 1/2 sum c H equals E[F(nu + d)] with
    d ~ N(0, C) exactly; the expectation here is a Gauss-Hermite quadrature."""
    rng = np.random.default_rng(seed)
    m = _quad_model(oracle, rng)
    nu = rng.uniform(0.005, 0.02, 2)
    A = rng.normal(size=(2, 2)) * 1e-3
    Cm = A @ A.T
    X = np.array([nu[0], nu[1], Cm[0, 0], Cm[0, 1], Cm[1, 1], 0, 0, 0])
    d = oracle.drift(m, X, 0.0, 0.0, 0.0)
    t, w = np.polynomial.hermite_e.hermegauss(8)
    Lc = np.linalg.cholesky(Cm)
    for p, idx in ((0, E), (1, I)):
        EF = 0.0
        for a in range(len(t)):
            for b in range(len(t)):
                x = nu + Lc @ np.array([t[a], t[b]])
                EF += w[a] * w[b] * _qF(m, p, x)
        EF /= (2 * np.pi)
        np.testing.assert_allclose(d[idx] * m.T, EF - nu[p], rtol=1e-10, atol=1e-16)


@pytest.mark.parametrize("seed", range(5))
def test_covariance_fixed_point_solves_lyapunov(oracle, seed):
    """Eq. (2) with a linear F at its fixed point nu* = F(nu*): the stationary
    covariance solves (J - I) C + C (J - I)^T + D = 0 (scipy's solver), where D is
    the finite-size term."""
    rng = np.random.default_rng(100 + seed)
    m = _quad_model(oracle, rng)
    for p in range(2):
        m.q_H[p][0] = m.q_H[p][1] = m.q_H[p][2] = 0.0
    J = np.array([[m.q_g[0][0], m.q_g[0][1]], [m.q_g[1][0], m.q_g[1][1]]]) * 0.4
    for p in range(2):
        m.q_g[p][0], m.q_g[p][1] = J[p]
    F0 = np.array(m.q_F0[:])
    nu = np.linalg.solve(np.eye(2) - J, F0)       # F(nu) = nu
    if np.any(nu <= 0) or np.any(np.linalg.eigvals(J - np.eye(2)).real >= 0):
        pytest.skip("draw has no stable positive fixed point")
    Nn = np.array([m.N_e, m.N_i])
    Dm = np.diag(nu * (1 / m.T - nu) / Nn)
    C = linalg.solve_continuous_lyapunov(J - np.eye(2), -Dm)
    X = np.array([nu[0], nu[1], C[0, 0], C[0, 1], C[1, 1], 0, 0, 0])
    d = oracle.drift(m, X, 0.0, 0.0, 0.0)
    scale = np.abs(C).max() / m.T
    assert np.all(np.abs(d[[CEE, CEI, CII]]) <= 1e-9 * scale)
    assert np.all(np.abs(d[[E, I]]) <= 1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_covariance_drift_outer_product_term(oracle, seed):
    """Eq. (2) at C = 0 with infinitely many neurons: T dC = (T dnu)(T dnu)^T,
    the outer product of the rate equation's own drift."""
    rng = np.random.default_rng(200 + seed)
    m = _quad_model(oracle, rng, N_big=True)
    nu = rng.uniform(0.001, 0.03, 2)
    d = oracle.drift(m, np.array([nu[0], nu[1], 0, 0, 0, 0, 0, 0.0]), 0.0, 0.0, 0.0)
    g = d[[E, I]] * m.T
    np.testing.assert_allclose(d[[CEE, CEI, CII]] * m.T, [g[0] * g[0], g[0] * g[1], g[1] * g[1]],
                               rtol=1e-12, atol=1e-20)


def test_finite_size_term_is_binomial_rate_variance(oracle):
    """Eq. (2) with a constant F = nu and C = 0 leaves only the finite-size term,
    which equals the variance of the empirical rate of N neurons each firing
    with probability F T in a window T (binomial)."""
    rng = np.random.default_rng(7)
    m = _quad_model(oracle, rng)
    for p in range(2):
        m.q_g[p][0] = m.q_g[p][1] = 0.0
        m.q_H[p][0] = m.q_H[p][1] = m.q_H[p][2] = 0.0
    F = np.array(m.q_F0[:])
    d = oracle.drift(m, np.array([F[0], F[1], 0, 0, 0, 0, 0, 0.0]), 0.0, 0.0, 0.0)
    for p, idx, N in ((0, CEE, m.N_e), (1, CII, m.N_i)):
        var = stats.binom(int(N), F[p] * m.T).var() / (N * m.T) ** 2
        np.testing.assert_allclose(d[idx] * m.T, var, rtol=1e-12)
    assert d[CEI] == 0.0


def test_adaptation_fixed_point_adex_form(oracle):
    """Eq. (3), AdEx form: at rest W* = tau_w b nu + a (mu_V - E_L), with mu_V
    evaluated at W* itself (solved with scipy)."""
    m = oracle.model()
    nu_e, nu_i, b, a = 0.004, 0.01, 40.0, 3.0
    X = np.array([nu_e, nu_i, 0, 0, 0, 0, 0, 0.0])

    def g(W):
        X[WE] = W
        return oracle.drift(m, X, 0.0, b, a)[WE]
    Wst = optimize.brentq(g, -1e4, 1e4, xtol=1e-13)
    xe = nu_e + m.cF_ee
    muV = oracle.tf(m, 0, xe, nu_i + m.cF_ei, Wst)[6]
    np.testing.assert_allclose(Wst, m.tau_w_e * b * nu_e + a * (muV - m.E_L_e), rtol=1e-10)


def test_heun_on_linear_ou_is_exact_ar1(oracle):
    """Eq. (4) under stochastic Heun: OU' = a OU + s z with
    a = 1 - h + h^2/2, h = dt/tau, s = (sigma/tau) sqrt(dt) (1 - h/2)."""
    m = oracle.model()
    dt = 0.1
    h = dt / m.tau_OU
    a = 1 - h + h * h / 2
    s = (m.sigma_OU / m.tau_OU) * np.sqrt(dt) * (1 - h / 2)
    rng = np.random.default_rng(3)
    X = np.array([0.004, 0.01, 0, 0, 0, 0, 0, 0.5e-3])
    for _ in range(50):
        z = rng.standard_normal()
        ou0 = X[OU]
        X, _ = oracle.step_region(m, X, 0.0, 0.0, 0.0, z, dt)
        np.testing.assert_allclose(X[OU], a * ou0 + s * z, rtol=1e-13, atol=1e-20)


def test_heun_is_second_order(oracle):
    """Noise-free single node: halving dt shrinks the error about 4x. The
    drive 0.3e-3 kHz keeps this trajectory inside the admissible set (the
    projection never acts), where the scheme's order is defined."""
    m = oracle.model(cF_ee=0.3e-3, cF_ie=0.3e-3)
    X0 = np.array([0.006, 0.012, 1e-6, 1e-6, 2e-6, 3.0, 0, 0])

    def integrate(dt, T=20.0):
        X = X0.copy()
        for _ in range(int(round(T / dt))):
            X, _ = oracle.step_region(m, X, 0.0, 30.0, 2.0, 0.0, dt)
        return X
    ref = integrate(0.0125)
    e1 = np.abs(integrate(0.2) - ref)[[E, I]].max()
    e2 = np.abs(integrate(0.1) - ref)[[E, I]].max()
    assert 3.6 < e1 / e2 < 4.4


def test_delays_are_numpy_rint(oracle):
    c = inputs.synthetic_connectome(68)
    for v in (1.0, 3.3, 4.0, 10.0):
        d = oracle.delays(c.tract_mm, v, 0.1)
        ref = np.maximum(np.rint(c.tract_mm / (float(np.float32(v)) * 0.1)), 1).astype(np.int32)
        assert np.array_equal(d, ref)
    # exact ties round half to even: v dt = 0.5, L/(v dt) = k + 1/2
    L = np.array([[0.0, 1.25], [1.75, 0.25]])
    assert oracle.delays(L, 4.0, 0.125).tolist() == [[1, 2], [4, 1]]


def test_row_normalisation(oracle):
    c = inputs.synthetic_connectome(20, seed=5)
    w = c.weights.copy()
    w[3, :] = 0.0
    W = oracle.normalise_rows(w)
    s = W.sum(1)
    assert np.allclose(np.delete(s, 3), 1.0, rtol=1e-14) and s[3] == 0.0
    k = 7
    nz = w[k] > 0
    assert np.allclose(W[k, nz] / w[k, nz], W[k, nz][0] / w[k, nz][0], rtol=1e-14)


def test_fc_and_statistics_against_numpy(oracle):
    rng = np.random.default_rng(11)
    n, ns = 12, 500
    base = rng.standard_normal((ns, 1))
    x = 0.004 + 1e-4 * (0.6 * base + rng.standard_normal((ns, n)))
    w = inputs.synthetic_connectome(n, seed=9).weights
    fc, st, flags = oracle.fc_stats(x, w)
    np.testing.assert_allclose(fc, np.corrcoef(x.T), rtol=0, atol=1e-12)
    iu = np.triu_indices(n, 1)
    np.testing.assert_allclose(st[0], fc[iu].mean(), rtol=1e-12)
    np.testing.assert_allclose(st[1], fc[iu].std(), rtol=1e-12)
    np.testing.assert_allclose(st[2], stats.pearsonr(fc[iu], w[iu])[0], rtol=1e-10)
    np.testing.assert_allclose(st[3], 1000 * x.mean(), rtol=1e-12)
    np.testing.assert_allclose(st[4], 1000 * x.std(0).mean(), rtol=1e-12)
    chi = np.sqrt(x.mean(1).var() / x.var(0).mean())
    np.testing.assert_allclose(st[5], chi, rtol=1e-12)
    assert flags == 0


def test_sync_index_limits(oracle):
    rng = np.random.default_rng(12)
    n, ns = 16, 20000
    w = inputs.synthetic_connectome(n, seed=9).weights
    same = np.repeat(rng.standard_normal((ns, 1)), n, 1)
    assert abs(oracle.fc_stats(same, w)[1][5] - 1.0) < 1e-12
    indep = rng.standard_normal((ns, n))
    assert abs(oracle.fc_stats(indep, w)[1][5] - 1 / np.sqrt(n)) < 0.02
    # a constant region: zero variance flag, its FC row is 0 off the diagonal
    x = indep.copy()
    x[:, 2] = 0.5
    fc, _, flags = oracle.fc_stats(x, w)
    assert flags & 4 and np.all(np.delete(fc[2], 2) == 0) and fc[2, 2] == 1.0


def test_silent_regions(oracle):
    """A region whose rate std is below the silence threshold counts as
    zero-variance; the other regions keep numpy's correlations."""
    rng = np.random.default_rng(13)
    n, ns = 10, 3000
    x = 0.004 + 1e-4 * rng.standard_normal((ns, n))
    x[:, 3] = 4e-11 + 1e-12 * rng.standard_normal(ns)       # std 1e-12 kHz: silent
    w = inputs.synthetic_connectome(n, seed=2).weights
    fc, st, flags = oracle.fc_stats(x, w, min_std=1e-9)
    keep = [k for k in range(n) if k != 3]
    np.testing.assert_allclose(fc[np.ix_(keep, keep)], np.corrcoef(x[:, keep].T), atol=1e-12)
    assert flags & 4 and fc[3, 3] == 1.0 and np.all(np.delete(fc[3], 3) == 0)
    fc0, _, flags0 = oracle.fc_stats(x, w, min_std=0.0)
    np.testing.assert_allclose(fc0, np.corrcoef(x.T), atol=1e-12)
    assert flags0 == 0
    # the silent region adds nothing to the population variance
    xs = x.copy()
    xs[:, 3] = 0.0
    chi = np.sqrt(xs.mean(1).var() / xs.var(0).mean())
    np.testing.assert_allclose(st[5], chi, rtol=1e-9)


def test_uncoupled_network_is_independent_nodes(oracle):
    """S = 0: every region follows the single-region stepper driven by its own
    Philox normal stream; no coupling leaks through."""
    m = oracle.model()
    conn = inputs.synthetic_connectome(6, seed=21)
    b = inputs._batch([0.0], [30.0], [2.0], [2.0])
    cfg = inputs.RunConfig(n_steps=60, n_trace_steps=60, seed=5)
    r = oracle.run(m, cfg, conn, b, inst_ids=[9], n_threads=1)
    for k in range(6):
        X = np.array([m.E_init, m.I_init, 0, 0, 0, 0, 0, 0.0])
        for n in range(60):
            X, _ = oracle.step_region(m, X, 0.0, 30.0, np.float32(2.0), oracle.normal(5, 9, n, k))
            np.testing.assert_array_equal(r["trace"][0, n, :, k], X)


@pytest.mark.parametrize("v", [1.0, 6.5])
def test_brute_force_tiny_network(oracle, v):
    """N = 3: the coupling S sum_j W_kj E_j(t - d_kj) computed in Python from a
    full history (rint delays, row-normalised weights, initial rate before t=0)
    reproduces the oracle's run step by step."""
    m = oracle.model()
    conn = inputs.synthetic_connectome(3, seed=4, density=1.0, len_lo=10, len_hi=40)
    S, be, ae = np.float32(0.37), np.float32(20.0), np.float32(1.0)
    b = inputs._batch([S], [be], [ae], [v])
    nsteps = 300
    cfg = inputs.RunConfig(n_steps=nsteps, n_trace_steps=nsteps, seed=2, transient_steps=100)
    r = oracle.run(m, cfg, conn, b, inst_ids=[4], n_threads=1)
    W = conn.weights / conn.weights.sum(1, keepdims=True)
    d = np.maximum(np.rint(conn.tract_mm / (float(np.float32(v)) * 0.1)), 1).astype(int)
    hist = [np.full(3, m.E_init)]
    X = np.tile(np.array([m.E_init, m.I_init, 0, 0, 0, 0, 0, 0.0])[:, None], (1, 3))
    for n in range(nsteps):
        Xn = X.copy()
        for k in range(3):
            c = sum(W[k, j] * hist[max(n - d[k, j], 0)][j] for j in range(3) if W[k, j] != 0)
            Xn[:, k], _ = oracle.step_region(m, X[:, k], float(S) * c, float(be), float(ae),
                                             oracle.normal(2, 4, n, k))
        X = Xn
        hist.append(X[E].copy())
        np.testing.assert_allclose(r["trace"][0, n], X, rtol=1e-12, atol=1e-18)
    # time averages: sample s is the mean of E after steps 10s+1 .. 10s+10
    Eh = np.array(hist[1:])
    smp = Eh.reshape(-1, 10, 3).mean(1)[10:]
    np.testing.assert_allclose(r["samples"][0], smp, rtol=1e-13)


def test_homogeneous_fixed_point_independent_of_speed(oracle):
    """Rows of W sum to 1, so with noise off the homogeneous state x* solving the
    single-node drift with coupling S E* is a fixed point of the network for any
    conduction speed."""
    m = oracle.model()
    S, be = 0.2, 5.0
    n = 10
    conn = inputs.synthetic_connectome(n, seed=3, density=0.6)
    assert np.all(conn.weights.sum(1) > 0)
    sc = np.array([1e-3, 1e-3, 1e-6, 1e-6, 1e-6, 1.0])

    def f(y):
        x = y * sc
        X = np.array([x[0], x[1], x[2], x[3], x[4], x[5], 0, 0])
        return oracle.drift(m, X, S * x[0], be, 0.0)[:6] * np.array([1, 1, 1e3, 1e3, 1e3, 1])
    sol = optimize.root(f, [4, 10, 2, 4, 10, 10], tol=1e-14, method="lm")
    assert sol.success and np.abs(f(sol.x)).max() < 1e-15
    x0 = np.array([*(sol.x * sc), 0.0, 0.0])
    m.E_init = x0[E]
    for v in (1.0, 10.0):
        b = inputs._batch([S], [be], [0.0], [v])
        cfg = inputs.RunConfig(n_steps=2000, transient_steps=0)
        r = oracle.run(m, cfg, conn, b, noise_off=True, init_state=x0, n_threads=1)
        np.testing.assert_allclose(r["final"][0], np.tile(x0[:, None], (1, n)), rtol=1e-6,
                                   atol=1e-15)


def test_inhibitory_adaptation_stays_zero(oracle):
    m = oracle.model()
    conn = inputs.synthetic_connectome(68)
    r = oracle.run(m, inputs.RunConfig(n_steps=500, n_trace_steps=500), conn,
                   inputs.grid_small().subset([0, 7]))
    assert np.all(r["trace"][:, :, WI, :] == 0.0)


def test_instance_parameters_equal_model_parameters(oracle):
    """The per-instance sweep axes (noise weight, tau_w_e, external drives) act
    exactly as the same values in the model: two instances with their own values
    reproduce, bit for bit, runs of models that carry those values."""
    conn = inputs.synthetic_connectome(6, seed=11)
    cfg = inputs.RunConfig(n_steps=300, transient_steps=0, n_trace_steps=300)
    b = inputs.grid_small().subset([1, 6])
    vals = [dict(w_noise=3e-4, tau_w_e=300.0, cF_ee=4e-4, cF_ei=1e-4, cF_ie=3e-4, cF_ii=0.0),
            dict(w_noise=1e-9, tau_w_e=700.0, cF_ee=3e-4, cF_ei=5e-4, cF_ie=5e-4, cF_ii=2e-4)]
    b.extra = {k: np.array([v[k] for v in vals]) for k in vals[0]}
    r = oracle.run(oracle.model("literature-B"), cfg, conn, b, n_threads=1)
    for q in range(2):
        m = oracle.model("literature-B", **vals[q])
        one = b.subset([q])
        one.extra = {}
        r1 = oracle.run(m, cfg, conn, one, inst_ids=[q], n_threads=1)
        assert np.array_equal(r["trace"][q], r1["trace"][0])
        assert np.array_equal(r["fc"][q], r1["fc"][0])
    # and they matter: the run differs from the default model's
    b0 = b.subset([0, 1])
    b0.extra = {}
    r0 = oracle.run(oracle.model("literature-B"), cfg, conn, b0, n_threads=1)
    assert not np.array_equal(r["trace"], r0["trace"])


@pytest.mark.parametrize("integrator", [0, 1])
def test_anchored_steps_reproduce_the_run(oracle, integrator):
    """Each step re-anchored on the oracle's own trajectory is that run's step,
    bit for bit (coupling from the trace's rates, the initial rate before t =
    0, the instance's own normals), for both integrators and per-instance
    Table 4 parameters; a trace changed at one step changes only the steps
    that read it."""
    conn = inputs.synthetic_connectome(20, seed=5, len_lo=2.0, len_hi=12.0)
    batch = inputs.grid_table4(np.array([5, 70000, 200001]))
    batch.v[:] = np.array([2.0, 3.5, 6.0], np.float32)
    cfg = inputs.RunConfig(n_steps=240, transient_steps=0, n_trace_steps=240, seed=9)
    m = oracle.model()
    ref = oracle.run(m, cfg, conn, batch, integrator=integrator)
    for q in range(len(batch)):
        out, _ = oracle.anchored_steps(m, cfg, conn, batch, q, ref["trace"][q], integrator=integrator)
        assert np.array_equal(out, ref["trace"][q])
    # a planted change of one region's rate after step 100: step 101 of that
    # region moves (its own state), and no region's step before its delay
    tr = ref["trace"][0].copy()
    tr[100, E, 3] *= 1.001
    out, _ = oracle.anchored_steps(m, cfg, conn, batch, 0, tr, integrator=integrator)
    diff = np.nonzero(np.any(out != ref["trace"][0], axis=1))
    steps, regions = diff
    assert 101 in steps[regions == 3]
    d = oracle.delays(conn.tract_mm, batch.v[0], cfg.dt_ms)
    W = conn.weights
    for s_, k in zip(steps, regions):
        assert s_ == 101 and k == 3 or (W[k, 3] != 0 and s_ == 101 + d[k, 3]), (s_, k)
