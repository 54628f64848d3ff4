"""Pins of the analysis-metric oracle (oracle/analysis.py, Section 2.6 and
Table 2) against independent library routines, closed forms and brute force."""
import numpy as np
import pytest
import scipy.signal

from oracle import analysis as A


def test_window_length():
    assert A.analysis_window(9000) == 8192
    assert A.analysis_window(8192) == 8192
    assert A.analysis_window(300) == 256
    assert A.analysis_window(1) == 1
    assert A.analysis_window(9000, 4096) == 4096
    assert A.analysis_window(50000) == 16384
    with pytest.raises(ValueError):
        A.analysis_window(9000, 3000)
    with pytest.raises(ValueError):
        A.analysis_window(1000, 2048)


@pytest.mark.parametrize("N,L", [(8192, 1024), (1000, 64), (256, 256), (300, 16)])
def test_welch_matches_scipy(N, L):
    rng = np.random.default_rng(N + L)
    x = 5.0 + np.cumsum(rng.standard_normal(N)) * 0.1 + rng.standard_normal(N)
    fs = 1000.0
    f, P = scipy.signal.welch(x, fs=fs, window="hann", nperseg=L, noverlap=L // 2,
                              detrend="constant", scaling="density", return_onesided=True,
                              average="mean")
    mine = A.welch_psd(x, fs, L)
    np.testing.assert_allclose(mine, P, rtol=1e-11, atol=1e-14 * P.max())
    np.testing.assert_allclose(A.psd_freqs(fs, L), f, rtol=0, atol=1e-12)


def test_welch_sinusoid_closed_form():
    """A cos(2 pi m t / L) over whole segments: with the periodic Hann window
    (sum w = L/2, sum w^2 = 3L/8) the segment DFT is A L / 4 at bin m and
    -A L / 8 at m +- 1, so P_m = A^2 L / (3 fs) and P_{m+-1} = A^2 L / (12 fs);
    the constant offset is removed."""
    L, m, Amp, fs = 256, 10, 3.0, 1000.0
    t = np.arange(4 * L)
    x = 7.0 + Amp * np.cos(2 * np.pi * m * t / L)
    P = A.welch_psd(x, fs, L)
    assert P[m] == pytest.approx(Amp ** 2 * L / (3 * fs), rel=1e-12)
    assert P[m - 1] == pytest.approx(Amp ** 2 * L / (12 * fs), rel=1e-12)
    assert P[m + 1] == pytest.approx(Amp ** 2 * L / (12 * fs), rel=1e-12)
    others = np.delete(P, [m - 1, m, m + 1])
    assert others.max() < 1e-20 * P[m] + 1e-25
    f, amp, b = A.psd_peak(P, fs, L)
    assert b == m and f == pytest.approx(m * fs / L) and amp == P[m]


def test_peak_ties_and_dc():
    P = np.array([100.0, 1.0, 5.0, 5.0, 2.0])      # DC is never the peak; ties go low
    f, amp, b = A.psd_peak(P, 8.0, 8)
    assert b == 2 and amp == 5.0 and f == 2.0


def test_fit_exact_power_law():
    fs, L = 1000.0, 1024
    f = A.psd_freqs(fs, L)
    a_true, b_true = 1.7, 42.0
    P = np.zeros_like(f)
    P[1:] = b_true / f[1:] ** a_true
    a, lb, nb = A.psd_fit(P, fs, L, 1.0, 100.0)
    assert a == pytest.approx(a_true, abs=1e-12)
    assert lb == pytest.approx(np.log10(b_true), abs=1e-12)
    assert nb == int(np.sum((f >= 1.0) & (f <= 100.0)))


def test_fit_skips_zero_bins_and_degenerate_band():
    fs, L = 1000.0, 64
    f = A.psd_freqs(fs, L)
    P = np.zeros_like(f)
    P[1:] = 3.0 / f[1:] ** 2
    P[3] = 0.0
    a, lb, nb = A.psd_fit(P, fs, L, 10.0, 200.0)
    assert a == pytest.approx(2.0, abs=1e-12) and lb == pytest.approx(np.log10(3.0), abs=1e-12)
    assert nb == int(np.sum((f >= 10.0) & (f <= 200.0))) - 1
    assert A.psd_fit(np.zeros_like(f), fs, L, 10.0, 200.0) == (0.0, 0.0, 0)
    assert A.psd_fit(P, fs, L, 20.0, 21.0) == (0.0, 0.0, 0)        # no bin in the band


@pytest.mark.parametrize("N", [16, 256, 8192])
def test_analytic_signal_matches_scipy(N):
    rng = np.random.default_rng(N)
    x = 3.0 + rng.standard_normal(N)
    z = A.analytic_signal(x)
    ref = scipy.signal.hilbert(x - x.mean())
    np.testing.assert_allclose(z, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(z.real, x - x.mean(), rtol=0, atol=1e-12)


def test_analytic_signal_cosine_closed_form():
    N = 1024
    t = np.arange(N)
    for m, ph in [(1, 0.3), (37, -1.2), (N // 2 - 1, 2.0)]:
        w = 2 * np.pi * m * t / N + ph
        z = A.analytic_signal(5.0 + np.cos(w))
        np.testing.assert_allclose(z, np.exp(1j * w), rtol=0, atol=1e-12)


def test_pli_sign_equals_phase_difference_definition():
    """Brute force: sign(Im(z_k conj z_l)) against sign(sin(angle z_k - angle z_l))."""
    rng = np.random.default_rng(3)
    Z = rng.standard_normal((5, 64)) + 1j * rng.standard_normal((5, 64))
    P = A.pli_matrix(Z)
    ph = np.angle(Z)
    for k in range(5):
        for l in range(5):
            if k == l:
                assert P[k, l] == 0.0
                continue
            s = np.sin(ph[k] - ph[l])
            assert np.all(np.abs(s) > 1e-9)
            assert P[k, l] == pytest.approx(abs(np.sign(s).sum()) / 64, abs=1e-15)


def test_pli_closed_forms():
    N = 2048
    t = np.arange(N)
    w = 2 * np.pi * 20 * t / N
    sig = [np.cos(w), np.cos(w - 0.7), np.cos(w + 2.5), np.cos(w)]
    Z = np.stack([A.analytic_signal(s) for s in sig])
    P = A.pli_matrix(Z)
    assert P[0, 1] == pytest.approx(1.0) and P[0, 2] == pytest.approx(1.0)
    assert P[1, 2] == pytest.approx(1.0)
    # identical signals: Im(z conj z) = 0 exactly
    assert P[0, 3] == 0.0
    # independent noise: |mean sign| of order 1/sqrt(N)
    rng = np.random.default_rng(0)
    Zn = np.stack([A.analytic_signal(rng.standard_normal(N)) for _ in range(6)])
    Pn = A.pli_matrix(Zn)
    assert A.mean_upper(Pn) < 4.0 / np.sqrt(N)
    assert A.mean_upper(np.zeros((1, 1))) == 0.0


def _ud_state_machine(x, band, min_range):
    """Sample-by-sample Schmitt trigger (brute force)."""
    x = np.asarray(x, np.float32)
    th = A.ud_thresholds(x, band, min_range)
    if th is None:
        return 0, 0, 0, 0
    up, dn = th
    state, entered, real_entry = 0, -1, False
    su = nu = sd = nd = 0
    for t, v in enumerate(x):
        new = 1 if v > up else (-1 if v < dn else state)
        if new != state:
            if real_entry:              # the state just left began at a transition
                if state > 0:
                    su += t - entered
                    nu += 1
                else:
                    sd += t - entered
                    nd += 1
            real_entry = state != 0     # leaving the unknown start is no transition
            state, entered = new, t
    return su, nu, sd, nd


def test_ud_square_wave_exact():
    # Down 300 samples at 0.5 Hz, Up 100 at 20 Hz, repeated; noise inside the band
    rng = np.random.default_rng(1)
    seg = np.concatenate([np.full(300, 0.0005), np.full(100, 0.020)])
    x = np.tile(seg, 6)[50:].astype(np.float32)     # starts inside a Down state
    x = x + (rng.standard_normal(len(x)) * 1e-4).astype(np.float32)
    su, nu, sd, nd = A.ud_durations(x, 0.1, 1e-3)
    # complete states: Up 100 x 6, Down 300 x 5 (first Down cut by the window start)
    assert (nu, nd) == (5, 5) and su == 500 and sd == 1500
    assert _ud_state_machine(x, 0.1, 1e-3) == (su, nu, sd, nd)


def test_ud_hysteresis_and_degenerate_cases():
    x = np.full(400, 0.001, np.float32)
    x[100:200] = 0.021
    x[150] = 0.0105          # dips past the centre but not below centre - band
    x[300] = 0.012           # rises past the centre but not above centre + band
    # states: Down (cut), Up 100-200, Down 200-end (cut) -> one Up of 100
    assert A.ud_durations(x, 0.1, 1e-3) == (100, 1, 0, 0)
    assert A.ud_durations(np.full(64, 0.004, np.float32)) == (0, 0, 0, 0)   # flat
    y = (0.004 + 1e-4 * np.sin(np.arange(512) / 5.0)).astype(np.float32)
    assert A.ud_durations(y, 0.1, 1e-3) == (0, 0, 0, 0)                     # range < 1 Hz


def test_ud_vectorised_equals_state_machine():
    rng = np.random.default_rng(7)
    for trial in range(200):
        N = int(rng.integers(2, 80))
        x = (rng.random(N) ** 3 * 0.03).astype(np.float32)
        band = float(rng.choice([0.0, 0.05, 0.1, 0.3]))
        assert A.ud_durations(x, band, 1e-3) == _ud_state_machine(x, band, 1e-3), trial


def test_analyze_instance_flat_and_mixed():
    n_s, n = 600, 4
    t = np.arange(n_s)
    S = np.zeros((n_s, n), np.float32)
    S[:, 0] = 0.004                                          # flat
    S[:, 1] = 0.004 + 0.002 * np.cos(2 * np.pi * 20 * t / 512)   # bin 20 of the window
    S[:, 2] = 0.004 + 0.002 * np.cos(2 * np.pi * 20 * t / 512 - 1.0)
    S[:, 3] = np.where((t // 100) % 2 == 0, 0.0005, 0.02)
    r = A.analyze_instance(S, 1.0)
    assert r["window"] == 512 and r["segment"] == 512
    assert np.all(r["psd"][0] == 0.0)
    assert np.all(r["analytic"][0] == 0.0)
    assert r["pli"][0].max() == 0.0
    assert r["pli"][1, 2] == pytest.approx(1.0)
    assert r["ud"][0].tolist() == [0, 0, 0, 0]
    su, nu, sd, nd = r["ud"][3].tolist()
    assert nu >= 1 and nd >= 1 and su == 100 * nu and sd == 100 * nd     # 100-ms states
    assert r["ud_up_count"] == r["ud"][:, 1].sum()
    assert r["ud_up_ms"] == pytest.approx(r["ud"][:, 0].sum() / r["ud"][:, 1].sum())
    # the instance spectrum is the mean of the region spectra
    np.testing.assert_allclose(r["mean_psd"], r["psd"].mean(axis=0), rtol=1e-15)


def test_fc_fitness_against_scipy_and_invariances():
    import scipy.stats
    rng = np.random.default_rng(5)
    n = 20
    F = rng.uniform(-0.2, 0.9, (n, n))
    F = (F + F.T) / 2
    np.fill_diagonal(F, 1.0)
    R = rng.uniform(-0.2, 0.9, (n, n))
    R = (R + R.T) / 2
    np.fill_diagonal(R, 7.0)                               # the diagonal takes no part
    iu = np.triu_indices(n, 1)
    want = scipy.stats.pearsonr(F[iu], R[iu])[0]
    assert A.fc_fitness(F, R) == pytest.approx(want, abs=1e-13)
    assert A.fc_fitness(F, 3.0 * R - 2.0) == pytest.approx(want, abs=1e-13)
    assert A.fc_fitness(F, -R) == pytest.approx(-want, abs=1e-13)
    assert A.fc_fitness(F, F) == pytest.approx(1.0, abs=1e-14)
    assert A.fc_fitness(np.eye(n), R) == 0.0               # no variance off the diagonal
    assert A.fc_fitness(np.eye(1), np.eye(1)) == 0.0


def test_top_k_definition():
    s = np.array([0.5, 2.0, 2.0, -1.0, 2.0, 0.5])
    assert A.top_k(s, 4).tolist() == [1, 2, 4, 0]
    assert A.top_k(s, 0).tolist() == []
    rng = np.random.default_rng(1)
    for _ in range(50):
        v = rng.integers(0, 5, 40).astype(float)
        k = int(rng.integers(1, 40))
        got = A.top_k(v, k)
        # brute force: sort pairs (-value, index)
        want = [i for _, i in sorted((-v[i], i) for i in range(40))][:k]
        assert got.tolist() == want


def test_bold_rest_and_fixed_point():
    """At rest (z = 0) everything stays at (0, 1, 1, 1) and the BOLD is 0; under
    a constant input the Runge-Kutta run converges to the closed-form fixed
    point f = 1 + z/gamma, v = f^alpha, q = v (1 - (1 - E0)^(1/f)) / E0."""
    z0 = np.zeros((3000, 2))
    assert np.all(A.bold_series(z0, 1.0) == 0.0)
    z = np.full((12000, 2), 0.004)                     # 4 Hz for 120 s in 10-ms samples
    y = A.bold_series(z, 10.0, tr_ms=1000.0)
    x_star, y_star = A.bold_fixed_point(0.004)
    assert y.shape == (120, 2)
    assert y[-1, 0] == pytest.approx(y_star, rel=1e-6)
    # the fixed point solves the equations
    np.testing.assert_allclose(A.bold_rhs(x_star[:, None], 0.004, A.BOLD_DEFAULTS)[:, 0], 0.0,
                               atol=1e-15)


def test_bold_rk4_is_fourth_order():
    """Halving the step cuts the error of RK4 by 16 (input held piecewise
    constant: a smooth input sampled finely enough that the hold error stays
    below the integration error is not needed -- the same held input is used
    at both steps by repeating each sample)."""
    rng = np.random.default_rng(2)
    base = 0.004 + 0.003 * np.sin(np.arange(400) / 15.0)[:, None] * np.ones((1, 3)) \
        + 0.0005 * rng.standard_normal((400, 3))
    def run(rep, period):
        z = np.repeat(base, rep, axis=0)
        return A.bold_series(z, period, tr_ms=400.0 * rep * period / 4)
    ref = run(64, 100.0 / 64)
    e1 = np.abs(run(1, 100.0) - ref).max()
    e2 = np.abs(run(2, 50.0) - ref).max()
    assert 12 < e1 / e2 < 20


def test_bold_sampling_times():
    z = np.full((5000, 1), 0.002)
    y = A.bold_series(z, 1.0, tr_ms=720.0)
    assert y.shape == (6, 1)                           # 0.72 .. 4.32 s
    y2 = A.bold_series(z[:720 * 3], 1.0, tr_ms=720.0)
    np.testing.assert_array_equal(y[:3], y2)
