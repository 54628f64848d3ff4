"""Seeded synthetic inputs for the TVB-AdEx sweep path.

This module is the ONLY code shared by the GPU library's callers and the CPU
oracle's tests. It draws random numbers and lays out parameter grids; it holds
none of the method's arithmetic (no weight normalisation, no delays, no model
equations).

Stand-ins: the paper's 68-region human connectome (Section 2.4, the ``-cf``
flag) is not available, so a synthetic connectome with the same region count
and the same role (symmetric weights, tract lengths in mm) replaces it. The
sweep axes follow Section 2.3 (one parameter combination per instance, grids of
equally spaced values per axis) and the parameter ranges of Table 4.
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np

# Region counts of the three size classes and the generator seed of each.
CONNECTOME_SEEDS = {68: 0, 84: 1, 200: 2}

# Box of the swept parameters (S, b_e [pA], a_e [nS], v [m/s]).
SWEEP_BOX = {"S": (0.0, 0.5), "b_e": (0.0, 120.0), "a_e": (0.0, 8.0), "v": (1.0, 10.0)}


@dataclasses.dataclass
class Connectome:
    """Raw structural connectivity of one synthetic brain.

    weights: [n, n] float64, symmetric, zero diagonal, raw (not normalised).
    tract_mm: [n, n] float64, symmetric, zero diagonal, lengths in mm.
    """

    weights: np.ndarray
    tract_mm: np.ndarray

    @property
    def n(self) -> int:
        return int(self.weights.shape[0])


def synthetic_connectome(n: int = 68, seed: int | None = None, density: float = 0.2,
                         lognorm_mu: float = -2.0, lognorm_sigma: float = 1.0,
                         len_lo: float = 10.0, len_hi: float = 200.0) -> Connectome:
    """Symmetric random connectome: each pair i<j is an edge with probability
    ``density``; edge weights are LogNormal(mu, sigma); tract lengths are
    U(len_lo, len_hi) mm for every pair. Draw order is fixed: edge mask, then
    weights, then lengths, each as a full [n, n] draw whose upper triangle is
    mirrored."""
    if seed is None:
        seed = CONNECTOME_SEEDS.get(n, n)
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    w = rng.lognormal(lognorm_mu, lognorm_sigma, (n, n))
    L = rng.uniform(len_lo, len_hi, (n, n))
    iu = np.triu_indices(n, 1)
    W = np.zeros((n, n))
    W[iu] = np.where(mask[iu], w[iu], 0.0)
    W = W + W.T
    T = np.zeros((n, n))
    T[iu] = L[iu]
    T = T + T.T
    return Connectome(weights=W, tract_mm=T)


@dataclasses.dataclass
class Batch:
    """One parameter combination per instance, FP32 as the library takes them."""

    S: np.ndarray
    b_e: np.ndarray
    a_e: np.ndarray
    v: np.ndarray
    conn: np.ndarray  # int32 connectome index per instance
    # further per-instance model parameters (Table 4 axes), name -> float64 array:
    # w_noise, tau_w_e, cF_ee, cF_ei, cF_ie, cF_ii; absent names take the model's value
    extra: dict = dataclasses.field(default_factory=dict)

    def __len__(self) -> int:
        return int(self.S.shape[0])

    def subset(self, idx) -> "Batch":
        idx = np.asarray(idx)
        return Batch(self.S[idx], self.b_e[idx], self.a_e[idx], self.v[idx], self.conn[idx],
                     {k: np.asarray(v)[idx] for k, v in self.extra.items()})


def _batch(S, b_e, a_e, v, conn=None) -> Batch:
    S = np.asarray(S, np.float32)
    n = S.shape[0]
    conn = np.zeros(n, np.int32) if conn is None else np.asarray(conn, np.int32)
    return Batch(S, np.asarray(b_e, np.float32), np.asarray(a_e, np.float32),
                 np.asarray(v, np.float32), conn)


def grid_small() -> Batch:
    """8 combos: S in {0.1, 0.3} x b_e in {0, 60} x a_e in {0, 4}, v = 4 m/s
    (S outermost, a_e innermost)."""
    rows = list(itertools.product([0.1, 0.3], [0.0, 60.0], [0.0, 4.0]))
    S, b, a = (np.array(c) for c in zip(*rows))
    return _batch(S, b, a, np.full(len(rows), 4.0))


def grid_uniform(n_s: int = 64, n_b: int = 64, v: float = 4.0) -> Batch:
    """n_s x n_b inclusive linspace over S in [0, 0.5] x b_e in [0, 120] with
    a_e = 0 and one conduction speed (S outermost)."""
    S = np.linspace(*SWEEP_BOX["S"], n_s)
    b = np.linspace(*SWEEP_BOX["b_e"], n_b)
    SS, BB = np.meshgrid(S, b, indexing="ij")
    n = SS.size
    return _batch(SS.ravel(), BB.ravel(), np.zeros(n), np.full(n, v))


def grid_uneven(n_inst: int = 8192, seed: int = 3, sizes=(68, 84, 200)) -> Batch:
    """Mixed batch: region-count classes in equal thirds (shuffled), v ~ U(1, 10),
    S, b_e, a_e uniform over the sweep box. ``conn`` indexes ``sizes``."""
    rng = np.random.default_rng(seed)
    k = len(sizes)
    cls = np.repeat(np.arange(k), -(-n_inst // k))[:n_inst]
    rng.shuffle(cls)
    u = rng.random((n_inst, 4))
    lo = np.array([SWEEP_BOX[a][0] for a in ("S", "b_e", "a_e", "v")])
    hi = np.array([SWEEP_BOX[a][1] for a in ("S", "b_e", "a_e", "v")])
    p = lo + u * (hi - lo)
    return _batch(p[:, 0], p[:, 1], p[:, 2], p[:, 3], cls)


def sample_box(n: int = 32768, seed: int = 4) -> Batch:
    """Uniform random points in the 4-D sweep box (surrogate training set)."""
    rng = np.random.default_rng(seed)
    u = rng.random((n, 4))
    lo = np.array([SWEEP_BOX[a][0] for a in ("S", "b_e", "a_e", "v")])
    hi = np.array([SWEEP_BOX[a][1] for a in ("S", "b_e", "a_e", "v")])
    p = lo + u * (hi - lo)
    return _batch(p[:, 0], p[:, 1], p[:, 2], p[:, 3])


def grid_4d(res: int = 32) -> Batch:
    """res^4 inclusive linspace grid over the sweep box (S outermost, v innermost)."""
    axes = [np.linspace(*SWEEP_BOX[a], res) for a in ("S", "b_e", "a_e", "v")]
    G = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 4)
    return _batch(G[:, 0], G[:, 1], G[:, 2], G[:, 3])


MLP_SHAPES = (("W1", (128, 4)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
              ("W3", (6, 128)), ("b3", (6,)))


def mlp_init_params(seed: int = 0) -> np.ndarray:
    """Initial surrogate parameters (W1, b1, W2, b2, W3, b3 concatenated,
    row-major), each uniform in +-1/sqrt(fan_in), as float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in MLP_SHAPES:
        fan_in = {"W1": 4, "b1": 4, "W2": 128, "b2": 128, "W3": 128, "b3": 128}[name]
        b = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-b, b, shape).ravel())
    return np.concatenate(parts).astype(np.float32)


@dataclasses.dataclass
class RunConfig:
    """Time axis of one sweep run. Steps of dt ms; a rate sample is the mean of
    ``tavg_steps`` consecutive steps; samples starting before
    ``transient_steps`` are dropped from the FC."""

    dt_ms: float = 0.1
    n_steps: int = 10000
    transient_steps: int = 0
    tavg_steps: int = 10
    seed: int = 0
    n_trace_steps: int = 0
    fc_min_std: float = 1e-9   # kHz: regions with a smaller rate std are silent

    @property
    def n_samples(self) -> int:
        return (self.n_steps - self.transient_steps) // self.tavg_steps


# Named workloads: (batch factory, region classes, run config).
RUN_SMALL = RunConfig(n_steps=10000, transient_steps=0)           # 1 s, no transient
RUN_UNIFORM = RunConfig(n_steps=100000, transient_steps=10000)    # 10 s, 1 s transient
RUN_UNEVEN = RunConfig(n_steps=50000, transient_steps=10000)      # 5 s, 1 s transient


def synthetic_rate_series(n_inst: int, n: int, n_samples: int, seed: int = 5,
                          period_ms: float = 1.0) -> np.ndarray:
    """Seeded stand-in for stored excitatory rate samples, [n_inst][n_samples][n]
    float32 in kHz, with the mix of behaviours the analysis metrics separate:
    Up/Down alternation (Down ~0.5 Hz, Up 8-30 Hz, exponential state lengths of
    tens to hundreds of ms), oscillations shared between regions with
    region-specific phase lags plus coloured noise, random-walk (1/f^2) noise,
    flat regions and regions whose range stays below 1 Hz."""
    rng = np.random.default_rng(seed)
    t_ms = np.arange(n_samples) * period_ms
    out = np.empty((n_inst, n_samples, n), np.float32)
    for i in range(n_inst):
        f0 = rng.uniform(2.0, 60.0)                       # shared rhythm of this instance (Hz)
        kind = rng.choice(5, size=n, p=[0.3, 0.35, 0.2, 0.05, 0.1])
        for k in range(n):
            if kind[k] == 0:                              # Up/Down
                x = np.empty(n_samples)
                pos, up = 0, bool(rng.integers(2))
                lo, hi = rng.uniform(2e-4, 8e-4), rng.uniform(8e-3, 3e-2)
                while pos < n_samples:
                    d = max(1, int(rng.exponential(rng.uniform(40, 400) / period_ms)))
                    x[pos:pos + d] = hi if up else lo
                    pos += d
                    up = not up
                x = x + rng.standard_normal(n_samples) * 3e-4 * rng.random()
            elif kind[k] == 1:                            # shared oscillation with a lag
                lag = rng.uniform(-np.pi, np.pi)
                amp = rng.uniform(5e-4, 5e-3)
                noise = np.cumsum(rng.standard_normal(n_samples)) * 2e-5
                x = 4e-3 + amp * np.cos(2 * np.pi * f0 * t_ms / 1000.0 + lag) + noise \
                    + rng.standard_normal(n_samples) * amp * 0.2
            elif kind[k] == 2:                            # random walk around a mean
                x = 5e-3 + np.cumsum(rng.standard_normal(n_samples)) * rng.uniform(1e-5, 1e-4)
            elif kind[k] == 3:                            # flat
                x = np.full(n_samples, rng.uniform(1e-3, 1e-2))
            else:                                         # small fluctuations (< 1 Hz range)
                x = 3.85e-3 + rng.standard_normal(n_samples) * 5e-5
            out[i, :, k] = np.maximum(x, 0.0)
    return out


# The paper's vast exploration (Table 4): ten axes with their ranges and
# resolutions (g is the coupling S; the weight noise scales the OU input).
TABLE4_AXES = (("S", 0.1, 0.9, 8), ("b_e", 0.0, 100.0, 8), ("w_noise", 1e-9, 1e-4, 4),
               ("v", 1.0, 7.0, 4), ("tau_w_e", 250.0, 750.0, 4), ("a_e", -10.0, 20.0, 4),
               ("cF_ee", 0.3e-3, 0.5e-3, 2), ("cF_ei", 0.0, 0.5e-3, 2),
               ("cF_ie", 0.3e-3, 0.5e-3, 2), ("cF_ii", 0.0, 0.5e-3, 2))


def grid_table4(idx=None) -> Batch:
    """Points of the ten-axis Table 4 grid (262,144 points; `idx` selects a
    subset by flat index, axis order as listed, last axis fastest). External
    drives are given in kHz as the model takes them."""
    axes = [np.linspace(lo, hi, n) for _, lo, hi, n in TABLE4_AXES]
    shape = tuple(len(a) for a in axes)
    total = int(np.prod(shape))
    idx = np.arange(total) if idx is None else np.asarray(idx, np.int64)
    coords = np.unravel_index(idx, shape)
    vals = {name: axes[d][coords[d]] for d, (name, _, _, _) in enumerate(TABLE4_AXES)}
    b = _batch(vals["S"], vals["b_e"], vals["a_e"], vals["v"])
    b.extra = {k: np.asarray(vals[k], np.float64)
               for k in ("w_noise", "tau_w_e", "cF_ee", "cF_ei", "cF_ie", "cF_ii")}
    return b
