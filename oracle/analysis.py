"""Plain FP64 oracle of the analysis metrics of Section 2.6 (Table 2), computed
from the stored excitatory rate samples of one instance: the power spectral
density with its peak and its fit to b / f^a, the phase lag index between
regions, and the durations of Up and Down states. (mean_FC, the fourth metric
of Table 2, is the FC mean of the main oracle.) Also the fitness against a
reference FC and the ranking of a grid search (Section 2.4), and the
Balloon-Windkessel BOLD signal the paper's GPU kernel computes (Section 2.4,
after Stephan et al. 2007).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the CPU-baseline leg of
``bench.py``; never by the product path. It shares no code with the GPU
library.

The paper names these metrics and gives the fitted law, log PSD = log(b / f^a);
the remaining definitions are readings:

* Analysis window: the last N_a samples of the post-transient series, N_a the
  largest power of two not above their number and 16384 (16.4 s at 1-ms
  samples), or a caller's power of two. Every metric uses the same window.
* PSD: Welch's average of modified periodograms per region -- segments of L
  samples (a power of two, default 1024) advancing by L/2, each with its own
  mean removed and multiplied by the periodic Hann window
  w[m] = (1 - cos(2 pi m / L)) / 2; one-sided density
  P[f] = c_f |X_f|^2 / (fs sum w^2), c_f = 2 except at f = 0 and f = L/2
  (c = 1); rates in Hz, so P in Hz^2/Hz. The instance spectrum is the mean over
  regions.
* psd_fmax_ampmax: the frequency bin with the largest instance spectrum among
  bins 1..L/2 (the lowest bin on ties) and that value.
* fit_psd_slope: least-squares line log10 P = log10 b - a log10 f over the bins
  with f_lo <= f <= f_hi and P > 0; (a, log10 b), or (0, 0) with no fitted bin
  count when fewer than two bins qualify.
* PLI: the phase lag index of Stam et al. (2007),
  PLI_kl = |mean_t sign(sin(phi_k(t) - phi_l(t)))|, with phi the phase of the
  analytic signal of the region's window with its mean removed (discrete
  analytic signal: DFT, bin 0 zeroed, bins 1..N/2-1 doubled, bin N/2 kept,
  negative bins zeroed, inverse DFT); sign(sin(phi_k - phi_l)) =
  sign(Im(z_k conj(z_l))), sign(0) = 0. mean_PLI: the mean over k < l.
* Up/Down states: per region on the stored single-precision rates (kHz),
  thresholds in single precision -- range r = max - min, centre
  theta = min + 0.5 r, half-band h = band * r; a sample above theta + h enters
  Up, below theta - h enters Down (hysteresis); regions with r < min_range have
  no states. A state's duration runs from the sample that entered it to the
  one that left it; the states cut by the window's ends are not counted.
  mean_UD_duration: the mean Up and the mean Down duration (ms) over every
  counted state of every region.
"""
from __future__ import annotations

import numpy as np

DEFAULT_SEGMENT = 1024
MAX_WINDOW = 16384
DEFAULT_FIT_BAND_HZ = (1.0, 100.0)
DEFAULT_UD_BAND = 0.1
DEFAULT_UD_MIN_RANGE_KHZ = 1e-3


def analysis_window(n_samples: int, window: int = 0) -> int:
    """Length N_a of the analysis window (a power of two <= n_samples)."""
    if window:
        if window & (window - 1) or window > n_samples:
            raise ValueError("window must be a power of two not above the sample count")
        return window
    if n_samples < 1:
        raise ValueError("no samples")
    return min(1 << (int(n_samples).bit_length() - 1), MAX_WINDOW)


def hann_periodic(L: int) -> np.ndarray:
    m = np.arange(L, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * m / L)


def welch_psd(x_hz: np.ndarray, fs_hz: float, L: int) -> np.ndarray:
    """Welch density of one series (FP64), bins 0..L/2."""
    x = np.asarray(x_hz, np.float64)
    N = len(x)
    if L > N:
        raise ValueError("segment longer than the series")
    w = hann_periodic(L)
    hop = L // 2
    n_seg = (N - L) // hop + 1
    acc = np.zeros(L // 2 + 1)
    for s in range(n_seg):
        seg = x[s * hop: s * hop + L]
        X = np.fft.rfft((seg - seg.mean()) * w)
        acc += X.real ** 2 + X.imag ** 2
    acc /= n_seg
    c = np.full(L // 2 + 1, 2.0)
    c[0] = 1.0
    c[-1] = 1.0
    return acc * c / (fs_hz * np.sum(w * w))


def psd_freqs(fs_hz: float, L: int) -> np.ndarray:
    return np.arange(L // 2 + 1) * (fs_hz / L)


def psd_peak(P: np.ndarray, fs_hz: float, L: int):
    """(f_max Hz, amplitude, bin) of the largest P among bins 1..L/2."""
    b = 1 + int(np.argmax(P[1:]))
    return b * fs_hz / L, float(P[b]), b


def psd_fit(P: np.ndarray, fs_hz: float, L: int, f_lo: float, f_hi: float):
    """Least squares log10 P = log10 b - a log10 f: (a, log10 b, bins used)."""
    f = psd_freqs(fs_hz, L)
    use = (f >= f_lo) & (f <= f_hi) & (P > 0) & (f > 0)
    if use.sum() < 2:
        return 0.0, 0.0, 0
    X = np.log10(f[use])
    Y = np.log10(P[use])
    xm, ym = X.mean(), Y.mean()
    slope = np.sum((X - xm) * (Y - ym)) / np.sum((X - xm) ** 2)
    return float(-slope), float(ym - slope * xm), int(use.sum())


def analytic_signal(x: np.ndarray) -> np.ndarray:
    """Discrete analytic signal of x with its mean removed (N even)."""
    x = np.asarray(x, np.float64)
    N = len(x)
    h = np.zeros(N)
    h[1:N // 2] = 2.0
    h[N // 2] = 1.0
    return np.fft.ifft(np.fft.fft(x) * h)


def pli_matrix(Z: np.ndarray) -> np.ndarray:
    """PLI_kl for analytic signals Z [n][N]; diagonal 0."""
    n, N = Z.shape
    P = np.zeros((n, n))
    for k in range(n):
        im = Z[k].imag[None, :] * Z[k + 1:].real - Z[k].real[None, :] * Z[k + 1:].imag
        P[k, k + 1:] = np.abs(np.sign(im).sum(axis=1)) / N
    return P + P.T


def pli_ambiguous(Z: np.ndarray, eps: float) -> np.ndarray:
    """Per pair, the samples whose sign decision an error of eps times each
    signal's rms magnitude could flip: |Im(z_k conj z_l)| <=
    eps (rms_k |z_l| + |z_k| rms_l)."""
    n, N = Z.shape
    mag = np.abs(Z)
    rms = np.sqrt(np.mean(mag ** 2, axis=1))
    A = np.zeros((n, n), np.int64)
    for k in range(n):
        im = Z[k].imag[None, :] * Z[k + 1:].real - Z[k].real[None, :] * Z[k + 1:].imag
        lim = eps * (rms[k] * mag[k + 1:] + mag[k][None, :] * rms[k + 1:, None])
        A[k, k + 1:] = (np.abs(im) <= lim).sum(axis=1)
    return A + A.T


def mean_upper(M: np.ndarray) -> float:
    n = M.shape[0]
    if n < 2:
        return 0.0
    iu = np.triu_indices(n, 1)
    return float(M[iu].mean())


def fc_fitness(fc: np.ndarray, ref: np.ndarray) -> float:
    """Fitness of a simulated FC against a reference FC (Section 2.4, the
    comparison with an externally obtained FC): the Pearson correlation of
    FC_kl and ref_kl over the pairs k < l; 0 when either has no variance."""
    n = fc.shape[0]
    iu = np.triu_indices(n, 1)
    a = np.asarray(fc, np.float64)[iu]
    b = np.asarray(ref, np.float64)[iu]
    if a.size == 0:
        return 0.0
    da, db = a - a.mean(), b - b.mean()
    va, vb = np.sum(da * da), np.sum(db * db)
    if not (va > 0 and vb > 0):
        return 0.0
    return float(np.sum(da * db) / np.sqrt(va * vb))


def top_k(score: np.ndarray, k: int) -> np.ndarray:
    """Indices of the k largest scores in decreasing order, ties by increasing
    index (the grid search's ranking)."""
    s = np.asarray(score, np.float64)
    order = np.lexsort((np.arange(len(s)), -s))
    return order[:k]


def ud_thresholds(x_khz: np.ndarray, band: float, min_range: float):
    """Single-precision thresholds (up, down) of one region, or None."""
    x = np.asarray(x_khz, np.float32)
    mn, mx = x.min(), x.max()
    r = np.float32(mx - mn)
    if not r >= np.float32(min_range):
        return None
    theta = np.float32(mn + np.float32(np.float32(0.5) * r))
    h = np.float32(np.float32(band) * r)
    return np.float32(theta + h), np.float32(theta - h)


def ud_durations(x_khz: np.ndarray, band: float = DEFAULT_UD_BAND,
                 min_range: float = DEFAULT_UD_MIN_RANGE_KHZ):
    """(sum of Up durations, Up count, sum of Down durations, Down count) in
    samples for one region."""
    th = ud_thresholds(x_khz, band, min_range)
    if th is None:
        return 0, 0, 0, 0
    up, dn = th
    x = np.asarray(x_khz, np.float32)
    c = np.where(x > up, 1, np.where(x < dn, -1, 0))
    nz = np.flatnonzero(c)
    if len(nz) == 0:
        return 0, 0, 0, 0
    cv = c[nz]
    change = np.flatnonzero(cv[1:] != cv[:-1]) + 1     # entries into a new state
    t = nz[change]
    kind = cv[change]
    dur = np.diff(t)                                    # states between two entries
    k = kind[:-1]
    return (int(dur[k > 0].sum()), int((k > 0).sum()),
            int(dur[k < 0].sum()), int((k < 0).sum()))


def analyze_instance(samples_khz: np.ndarray, period_ms: float, window: int = 0,
                     segment: int = 0, fit_band=DEFAULT_FIT_BAND_HZ,
                     ud_band: float = DEFAULT_UD_BAND,
                     ud_min_range: float = DEFAULT_UD_MIN_RANGE_KHZ,
                     with_ambiguity: float = 0.0) -> dict:
    """All metrics of one instance from its [n_samples][n] FP32 samples (kHz)."""
    S = np.asarray(samples_khz, np.float32)
    n_samples, n = S.shape
    Na = analysis_window(n_samples, window)
    L = segment or min(DEFAULT_SEGMENT, Na)
    if L & (L - 1) or L > Na or L < 8:
        raise ValueError("segment must be a power of two in [8, window]")
    W = S[n_samples - Na:]
    fs = 1000.0 / period_ms
    x_hz = W.astype(np.float64) * 1000.0
    psd = np.stack([welch_psd(x_hz[:, k], fs, L) for k in range(n)])
    mpsd = psd.mean(axis=0)
    fmax, amax, bmax = psd_peak(mpsd, fs, L)
    a, lb, nfit = psd_fit(mpsd, fs, L, fit_band[0], fit_band[1])
    Z = np.stack([analytic_signal(W[:, k].astype(np.float64)) for k in range(n)])
    pli = pli_matrix(Z)
    ud = np.array([ud_durations(W[:, k], ud_band, ud_min_range) for k in range(n)], np.int64)
    su, nu, sd, nd = (int(v) for v in ud.sum(axis=0))
    out = {
        "window": Na, "segment": L, "fs_hz": fs, "psd": psd, "mean_psd": mpsd,
        "psd_fmax_hz": fmax, "psd_ampmax": amax, "psd_peak_bin": bmax,
        "psd_slope_a": a, "psd_log10_b": lb, "psd_fit_bins": nfit,
        "analytic": Z, "pli": pli, "mean_pli": mean_upper(pli), "ud": ud,
        "ud_up_sum": su, "ud_up_count": nu, "ud_down_sum": sd, "ud_down_count": nd,
        "ud_up_ms": su * period_ms / nu if nu else 0.0,
        "ud_down_ms": sd * period_ms / nd if nd else 0.0,
    }
    if with_ambiguity:
        out["pli_ambiguous"] = pli_ambiguous(Z, with_ambiguity)
    return out


# Balloon-Windkessel haemodynamics (Friston et al. 2000, as compared in Stephan
# et al. 2007): time in s; kappa, gamma in 1/s; tau0 in s.
BOLD_DEFAULTS = dict(kappa=0.65, gamma=0.41, tau0=0.98, alpha=0.32, E0=0.34, V0=0.02,
                     k1=7 * 0.34, k2=2.0, k3=2 * 0.34 - 0.2, tr_ms=2000.0)


def bold_rhs(x, z, p):
    """d/dt of (s, f, v, q) for neural input z; x: [4, n]."""
    s, f, v, q = x
    vpow = v ** (1.0 / p["alpha"])
    ds = z - p["kappa"] * s - p["gamma"] * (f - 1.0)
    df = s
    dv = (f - vpow) / p["tau0"]
    dq = (f * (1.0 - (1.0 - p["E0"]) ** (1.0 / f)) / p["E0"] - vpow * q / v) / p["tau0"]
    return np.stack([ds, df, dv, dq])


def bold_signal(x, p):
    s, f, v, q = x
    return p["V0"] * (p["k1"] * (1.0 - q) + p["k2"] * (1.0 - q / v) + p["k3"] * (1.0 - v))


def bold_series(samples_khz: np.ndarray, period_ms: float, **over) -> np.ndarray:
    """BOLD of every region from its rate samples [ns][n] (kHz: the neural
    input z is the excitatory rate in the model's unit, held over each sample
    interval). Readings: classical Runge-Kutta (RK4) with the sample period as
    the step, from rest (s = 0, f = v = q = 1); the signal sampled at
    t = m TR, m = 1 .. floor(ns period / TR). Returns [n_tr][n]."""
    p = dict(BOLD_DEFAULTS, **over)
    z = np.asarray(samples_khz, np.float64)
    ns, n = z.shape
    h = period_ms / 1000.0
    x = np.zeros((4, n))
    x[1:] = 1.0
    steps_per_tr = p["tr_ms"] / period_ms
    n_tr = int(np.floor(ns * period_ms / p["tr_ms"] + 1e-9))
    out = np.zeros((n_tr, n))
    m = 0
    for t in range(ns):
        zt = z[t]
        k1 = bold_rhs(x, zt, p)
        k2 = bold_rhs(x + 0.5 * h * k1, zt, p)
        k3 = bold_rhs(x + 0.5 * h * k2, zt, p)
        k4 = bold_rhs(x + h * k3, zt, p)
        x = x + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        # after sample t the clock reads (t + 1) periods
        while m < n_tr and (t + 1) >= round((m + 1) * steps_per_tr):
            out[m] = bold_signal(x, p)
            m += 1
    return out


def bold_fixed_point(z: float, **over):
    """Steady state (s, f, v, q) and BOLD for a constant input z."""
    p = dict(BOLD_DEFAULTS, **over)
    f = 1.0 + z / p["gamma"]
    v = f ** p["alpha"]
    q = v * (1.0 - (1.0 - p["E0"]) ** (1.0 / f)) / p["E0"]
    x = np.array([0.0, f, v, q])
    return x, float(bold_signal(x, p))
