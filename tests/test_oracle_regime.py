"""Regime pins of the oracle (Section 3.2): the fixed points of the noise-free
single-node drift with all eight states and their Jacobian eigenvalues, the
pathological fixed point near 190 Hz (Section 3.2.5), the bistability at low
spike-frequency adaptation, the loss of the active fixed point under strong
adaptation, and the qualitative trends of Section 3.2.1 (synchrony rising with
adaptation and coupling over the sweep box; excitatory-rate variability rising
with adaptation over the box of the g x b_e figure).

A homogeneous network (rows of the weights sum to one) sits at a fixed point
of the single node whose coupling input is S times its own rate, so the scan
uses c = S E. Roots come from scipy's hybrid Powell solver (a library routine)
from a grid of starting points; eigenvalues from central differences of the
oracle's drift. Readings pinned here: the literature-B threshold polynomial,
external drives c_F = 0.5e-3 kHz (Table 4's upper value), noise amplitude 1e-6,
initial rates E = 4 Hz, I = 10 Hz.
"""
import numpy as np
import pytest
from scipy import optimize, stats

from paper_2311_13337_amd import inputs

E, I, CEE, CEI, CII, WE, WI, OU = range(8)


def _drift_c(oracle, m, X, S, b_e, a_e=0.0):
    return oracle.drift(m, X, S * X[E], b_e, a_e)


def fixed_points(oracle, m, S, b_e, a_e=0.0):
    """Roots of the noise-free single-node drift with c = S E (W_i = OU = 0),
    each with the eigenvalues of the 8x8 Jacobian there (c follows E)."""
    scale = np.array([1e3, 1e3, 1e6, 1e6, 1e6, 1.0])

    def f(y):
        X = np.array([*y, 0.0, 0.0])
        return _drift_c(oracle, m, X, S, b_e, a_e)[:6] * scale

    roots = []
    for E0 in np.logspace(-7, np.log10(0.3), 24):
        for I0 in np.logspace(-6, np.log10(0.5), 8):
            r = optimize.root(f, [E0, I0, 0, 0, 0, m.tau_w_e * b_e * E0], method="hybr",
                              options={"xtol": 1e-13})
            y = r.x
            if not r.success or np.max(np.abs(f(y))) > 1e-9:
                continue
            if not (0 <= y[0] <= 1 and 0 <= y[1] <= 1 and y[2] >= -1e-12 and y[4] >= -1e-12):
                continue
            if any(abs(y[0] - q[0]) <= 1e-9 + 1e-6 * abs(q[0]) for q, _ in roots):
                continue
            X = np.array([*y, 0.0, 0.0])
            J = np.zeros((8, 8))
            for j in range(8):
                h = 1e-7 * max(abs(X[j]), 1e-6)
                Xp, Xm = X.copy(), X.copy()
                Xp[j] += h
                Xm[j] -= h
                J[:, j] = (_drift_c(oracle, m, Xp, S, b_e, a_e) - _drift_c(oracle, m, Xm, S, b_e, a_e)) / (2 * h)
            roots.append((X, np.linalg.eigvals(J)))
    roots.sort(key=lambda q: q[0][E])
    return roots


def settle(oracle, m, S, b_e, E0, I0, steps, dt=0.1):
    """Noise-free single node with c = S E from rates (E0, I0), the other
    states at zero; returns the excitatory rate after every step."""
    X = np.array([E0, I0, 0, 0, 0, 0, 0, 0.0])
    out = np.empty(steps)
    for n in range(steps):
        X, _ = oracle.step_region(m, X, S * X[E], b_e, 0.0, 0.0, dt=dt)
        out[n] = X[E]
    return out


def test_fixed_point_scan_roots_and_eigenvalues(oracle):
    """The scan's roots are roots of the full drift, and the stable active
    state at b_e = 0 has the W_e relaxation -1/tau_w,e among its
    eigenvalues (W_e enters no other equation at a_e = 0)."""
    m = oracle.model()
    roots = fixed_points(oracle, m, 0.0, 0.0)
    assert roots
    for X, ev in roots:
        assert np.max(np.abs(_drift_c(oracle, m, X, 0.0, 0.0)[:5])) < 1e-11
    act = [(X, ev) for X, ev in roots if 1e-3 <= X[E] <= 1e-2]
    assert len(act) == 1
    X, ev = act[0]
    assert np.max(ev.real) < 0
    assert np.min(np.abs(ev - (-1.0 / m.tau_w_e))) < 1e-6
    # the isolated node's asynchronous state: 4.07 Hz excitatory, 9.9 Hz inhibitory
    assert 3.5e-3 < X[E] < 4.5e-3 and X[I] > X[E]


@pytest.mark.parametrize("S", [0.0, 0.3])
def test_active_state_stable_at_low_adaptation(oracle, S):
    """At b_e = 0 the node has a stable low-rate active (asynchronous) fixed
    point of a few Hz, with and without coupling."""
    m = oracle.model()
    stable = [X for X, ev in fixed_points(oracle, m, S, 0.0)
              if np.max(ev.real) < 0 and 1e-3 <= X[E] <= 2e-2]
    assert len(stable) == 1


@pytest.mark.parametrize("S", [0.0, 0.3])
def test_pathological_fixed_point_near_190_hz(oracle, S):
    """Section 3.2.5: a fixed point near 190 Hz attracts every start from
    50 Hz up (noise-free, b_e = 0), where the rates stay (the moment bounds of
    the projection are active there, so it is a fixed point of the projected
    flow rather than a root of the drift)."""
    m = oracle.model()
    ends = []
    for E0, I0 in ((0.05, 0.05), (0.19, 0.19), (0.25, 0.3)):
        tr = settle(oracle, m, S, 0.0, E0, I0, 15000)
        assert 0.185 < tr[-1] < 0.200
        # settled: the last 500 ms vary by less than 1e-9 kHz
        assert np.ptp(tr[-5000:]) < 1e-9
        ends.append(tr[-1])
    assert np.ptp(ends) < 1e-9


def test_bistability_at_low_adaptation(oracle):
    """b_e = 0, S = 0: the asynchronous state (from 4 Hz) and the ~190 Hz
    state (from 190 Hz) are both reached and both persist: two stable
    states of one node."""
    m = oracle.model()
    lo = settle(oracle, m, 0.0, 0.0, 0.004, 0.01, 15000)
    hi = settle(oracle, m, 0.0, 0.0, 0.19, 0.19, 15000)
    # (the active state relaxes on the adaptation time scale, tau_w = 500 ms)
    assert 3.5e-3 < lo[-1] < 4.5e-3 and np.ptp(lo[-5000:]) < 1e-5 * lo[-1]
    assert 0.185 < hi[-1] < 0.2 and np.ptp(hi[-5000:]) < 1e-9


@pytest.mark.parametrize("b_e", [60.0, 120.0])
def test_strong_adaptation_leaves_no_stable_active_state(oracle, b_e):
    """With b_e = 60 or 120 pA (S = 0) no root between 0.1 and 100 Hz is
    stable: adaptation destabilises the active state, and the noise-free node
    started at 4 Hz keeps oscillating (slow adaptation cycles) instead of
    settling."""
    m = oracle.model()
    for X, ev in fixed_points(oracle, m, 0.0, b_e):
        if 1e-4 <= X[E] <= 0.1:
            assert np.max(ev.real) > 0, (X[E], np.max(ev.real))
    tr = settle(oracle, m, 0.0, b_e, 0.004, 0.01, 40000)
    late = tr[-20000:]
    assert np.ptp(late) > 0.5 * np.max(late)


def _grid_stats(oracle, S, b_e, v, n_steps, extra=None):
    conn = inputs.synthetic_connectome(68)
    nn = len(S)
    bt = inputs.Batch(np.asarray(S, np.float32), np.asarray(b_e, np.float32),
                      np.zeros(nn, np.float32), np.full(nn, v, np.float32),
                      np.zeros(nn, np.int32), extra or {})
    cfg = inputs.RunConfig(n_steps=n_steps, transient_steps=10000)
    return oracle.run(oracle.model(), cfg, conn, bt)["stats"]


def test_synchrony_rises_with_adaptation_and_coupling(oracle):
    """Section 3.2.1: asynchronous activity at low adaptation, synchronous
    activity as adaptation and coupling grow. 6 x 6 grid over the sweep box
    (S in [0, 0.5], b_e in [0, 120] pA, v = 4 m/s), 3-s runs after a 1-s
    transient."""
    S, B = np.meshgrid(np.linspace(0, 0.5, 6), np.linspace(0, 120, 6), indexing="ij")
    st = _grid_stats(oracle, S.ravel(), B.ravel(), 4.0, 30000)
    sync, fcm, rstd = st[:, 5], st[:, 0], st[:, 4]
    silent = rstd < 1e-3
    assert silent.sum() <= 3
    # b_e = 0: asynchronous (Golomb index near 1/sqrt(68) = 0.12), FC near 0
    a0 = B.ravel() == 0
    assert np.all(sync[a0] < 0.2) and np.all(np.abs(fcm[a0]) < 0.1)
    # strong adaptation with coupling: synchronous
    strong = (B.ravel() >= 72) & (S.ravel() >= 0.2)
    assert np.median(sync[strong]) > 0.5 and np.median(fcm[strong]) > 0.3
    assert stats.spearmanr(B.ravel(), sync)[0] > 0.4
    assert stats.spearmanr(S.ravel()[~a0], sync[~a0])[0] > 0.2


def test_adaptation_raises_rate_variability_in_figure_box(oracle):
    """Section 3.2.1: over the g x b_e figure's box (g in [0.4, 0.9], b_e in
    [60, 120] pA, v = 3 m/s, tau_w = 417 ms) raising the adaptation raises
    the variability of the excitatory rate, and no point is silent."""
    S, B = np.meshgrid(np.linspace(0.4, 0.9, 6), np.linspace(60, 120, 6), indexing="ij")
    st = _grid_stats(oracle, S.ravel(), B.ravel(), 3.0, 30000, {"tau_w_e": np.full(36, 417.0)})
    rstd = st[:, 4]
    assert np.all(rstd > 1e-3)
    assert stats.spearmanr(B.ravel(), rstd)[0] > 0.3
