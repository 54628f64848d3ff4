"""Python shim over the plain FP64 C oracle (``adex_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of ``bench.py``; never by the product path. It shares no code
with the GPU library. See the header of ``adex_oracle.c`` for what it computes
and which passages of the paper each part follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "adex_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_adex.so")

PRESETS = {"literature-B": 0, "paper-T1": 1}
N_SV = 8
STATE_NAMES = ("E", "I", "C_ee", "C_ei", "C_ii", "W_e", "W_i", "OU")
STAT_NAMES = ("fc_mean", "fc_std", "fc_sc_corr", "rate_mean_hz", "rate_std_hz", "sync_index")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-D_GNU_SOURCE", "-shared", "-fPIC", "-o", tmp, _SRC,
                               "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


class Model(C.Structure):
    _fields_ = [(f, C.c_double) for f in (
        "C_m", "g_L", "E_e", "E_i", "Q_e", "Q_i", "tau_e", "tau_i", "K_e", "K_i", "N_e", "N_i",
        "T", "E_L_e", "E_L_i", "tau_w_e", "tau_w_i", "b_i", "a_i",
        "cF_ee", "cF_ei", "cF_ie", "cF_ii", "tau_OU", "sigma_OU", "w_noise",
        "muV0", "dmuV0", "sV0", "dsV0", "tN0", "dtN0", "rate_max", "E_init", "I_init",
        "x_floor")] + [
        ("P_e", C.c_double * 10), ("P_i", C.c_double * 10), ("tf_kind", C.c_int64),
        ("q_F0", C.c_double * 2), ("q_g", (C.c_double * 2) * 2), ("q_H", (C.c_double * 3) * 2)]

    def scalar_fields(self):
        return [f for f, t in self._fields_ if t is C.c_double]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f in self.scalar_fields()}
        d["P_e"] = list(self.P_e)
        d["P_i"] = list(self.P_i)
        return d


class RunCfg(C.Structure):
    _fields_ = [("dt", C.c_double), ("n_steps", C.c_int64), ("transient_steps", C.c_int64),
                ("tavg_steps", C.c_int64), ("n_trace_steps", C.c_int64), ("seed", C.c_uint32),
                ("integrator", C.c_int32), ("noise_off", C.c_int32), ("fc_min_std", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P = C.POINTER
        dp = np.ctypeslib.ndpointer(np.float64, flags="C")
        fp = np.ctypeslib.ndpointer(np.float32, flags="C")
        up = np.ctypeslib.ndpointer(np.uint32, flags="C")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C")
        L.oracle_model_size.restype = C.c_size_t
        L.oracle_model_preset.argtypes = [C.c_int, P(Model)]
        L.oracle_tf.argtypes = [P(Model), C.c_int, C.c_double, C.c_double, C.c_double, dp]
        L.oracle_drift.argtypes = [P(Model), dp, C.c_double, C.c_double, C.c_double, dp]
        L.oracle_philox4x32_10.argtypes = [up, up, up]
        L.oracle_normal.argtypes = [C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32]
        L.oracle_normal.restype = C.c_double
        L.oracle_normalise_rows.argtypes = [C.c_int, dp, dp]
        L.oracle_delays.argtypes = [C.c_int, dp, C.c_float, C.c_double, ip]
        L.oracle_fc_stats.argtypes = [C.c_int, C.c_int64, dp, dp, C.c_double, dp, dp]
        L.oracle_fc_stats.restype = C.c_uint32
        L.oracle_step_region.argtypes = [P(Model), C.c_int, C.c_double, dp, C.c_double, C.c_double,
                                         C.c_double, C.c_double]
        L.oracle_step_region.restype = C.c_uint32
        L.oracle_project.argtypes = [P(Model), dp]
        L.oracle_project.restype = C.c_uint32
        vp = C.c_void_p
        L.oracle_run.argtypes = [P(Model), P(RunCfg), C.c_int, dp, dp, C.c_int64, fp, fp, fp, fp,
                                 up, vp, vp, dp, vp, vp, vp, vp, up, C.c_int]
        L.oracle_anchored_steps.argtypes = [P(Model), P(RunCfg), C.c_int, dp, dp, C.c_float, C.c_float,
                                            C.c_float, C.c_float, C.c_uint32, vp, C.c_int64, dp, dp]
        L.oracle_anchored_steps.restype = C.c_uint32
        assert L.oracle_model_size() == C.sizeof(Model), "oracle model layout mismatch"
        _lib = L
    return _lib


def model(preset: str = "literature-B", **overrides) -> Model:
    m = Model()
    if lib().oracle_model_preset(PRESETS[preset], C.byref(m)) != 0:
        raise ValueError(preset)
    for k, v in overrides.items():
        if k in ("P_e", "P_i"):
            getattr(m, k)[:] = list(v)
        else:
            setattr(m, k, v)
    return m


def tf(m: Model, pop: int, xe: float, xi: float, W: float = 0.0) -> np.ndarray:
    """[F, dF/dxe, dF/dxi, d2F/dxe2, d2F/dxedxi, d2F/dxi2, muV, sigmaV, tauV, Vthre]."""
    out = np.zeros(10)
    lib().oracle_tf(C.byref(m), pop, xe, xi, W, out)
    return out


def drift(m: Model, X, c: float, b_e: float, a_e: float) -> np.ndarray:
    X = np.ascontiguousarray(X, np.float64)
    out = np.zeros(N_SV)
    lib().oracle_drift(C.byref(m), X, c, b_e, a_e, out)
    return out


def step_region(m: Model, X, c, b_e, a_e, z, dt=0.1, integrator=0):
    X = np.array(X, np.float64)
    flags = lib().oracle_step_region(C.byref(m), integrator, dt, X, c, b_e, a_e, z)
    return X, flags


def project(m: Model, X):
    """The admissible-state projection applied after each stage; returns
    (projected state, flag bits)."""
    X = np.array(X, np.float64)
    flags = lib().oracle_project(C.byref(m), X)
    return X, flags


def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def normal(seed: int, inst: int, n: int, k: int) -> float:
    return lib().oracle_normal(seed, inst, n, k)


def normalise_rows(w) -> np.ndarray:
    w = np.ascontiguousarray(w, np.float64)
    out = np.zeros_like(w)
    lib().oracle_normalise_rows(w.shape[0], w, out)
    return out


def delays(L, v: float, dt: float) -> np.ndarray:
    L = np.ascontiguousarray(L, np.float64)
    out = np.zeros(L.shape, np.int32)
    lib().oracle_delays(L.shape[0], L, float(np.float32(v)), dt, out)
    return out


def fc_stats(samples, w_raw, min_std=0.0):
    x = np.ascontiguousarray(samples, np.float64)
    w = np.ascontiguousarray(w_raw, np.float64)
    n = w.shape[0]
    fc = np.zeros((n, n))
    st = np.zeros(6)
    flags = lib().oracle_fc_stats(n, x.shape[0], x, w, min_std, fc, st)
    return fc, st, flags


def anchored_steps(m: Model, run_cfg, conn, batch, q: int, trace, inst_id=None, integrator=0,
                   noise_off=False):
    """The oracle's steps of instance q of ``batch`` each re-anchored on a given
    trajectory ``trace`` [steps, 8, n] (state after every step, e.g. another
    implementation's): out[n] is one oracle step from trace[n-1] (the initial
    state for n = 0), with the coupling from trace's excitatory rates and the
    instance's Philox normals. Returns (out [steps, 8, n], flags)."""
    tr = np.ascontiguousarray(trace, np.float64)
    nt = tr.shape[0]
    r = RunCfg(dt=run_cfg.dt_ms, n_steps=nt, transient_steps=0, tavg_steps=run_cfg.tavg_steps,
               n_trace_steps=nt, seed=run_cfg.seed, integrator=integrator,
               noise_off=1 if noise_off else 0, fc_min_std=getattr(run_cfg, "fc_min_std", 1e-9))
    extra = None
    if getattr(batch, "extra", None):
        names = ("w_noise", "tau_w_e", "cF_ee", "cF_ei", "cF_ie", "cF_ii")
        extra = np.array([batch.extra[k][q] if k in batch.extra else getattr(m, k) for k in names],
                         np.float64)
    out = np.zeros_like(tr)
    fl = lib().oracle_anchored_steps(
        C.byref(m), C.byref(r), conn.n, np.ascontiguousarray(conn.weights, np.float64),
        np.ascontiguousarray(conn.tract_mm, np.float64), float(batch.S[q]), float(batch.b_e[q]),
        float(batch.a_e[q]), float(batch.v[q]), int(q if inst_id is None else inst_id), _ptr(extra),
        nt, tr, out)
    return out, fl


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def run(m: Model, run_cfg, conn, batch, inst_ids=None, n_trace_steps=None, want_samples=True,
        want_fc=True, noise_off=False, integrator=0, init_state=None, n_threads=None):
    """Integrate every instance of ``batch`` on connectome ``conn``.

    run_cfg: an object with dt_ms, n_steps, transient_steps, tavg_steps, seed
    (and optionally n_trace_steps). Returns a dict of numpy arrays:
    final [inst, 8, n], samples [inst, ns, n], trace [inst, nt, 8, n],
    fc [inst, n, n], stats [inst, 6], flags [inst].
    """
    n = conn.n
    ni = len(batch)
    nt = run_cfg.n_trace_steps if n_trace_steps is None else n_trace_steps
    r = RunCfg(dt=run_cfg.dt_ms, n_steps=run_cfg.n_steps, transient_steps=run_cfg.transient_steps,
               tavg_steps=run_cfg.tavg_steps, n_trace_steps=nt, seed=run_cfg.seed,
               integrator=integrator, noise_off=1 if noise_off else 0,
               fc_min_std=getattr(run_cfg, "fc_min_std", 1e-9))
    ns = (run_cfg.n_steps - run_cfg.transient_steps) // run_cfg.tavg_steps
    ids = np.arange(ni, dtype=np.uint32) if inst_ids is None else np.asarray(inst_ids, np.uint32)
    out = {
        "final": np.zeros((ni, N_SV, n)),
        "samples": np.zeros((ni, max(ns, 0), n)) if want_samples else None,
        "trace": np.zeros((ni, nt, N_SV, n)) if nt > 0 else None,
        "fc": np.zeros((ni, n, n)) if want_fc else None,
        "stats": np.zeros((ni, 6)) if want_fc else None,
        "flags": np.zeros(ni, np.uint32),
    }
    init = None if init_state is None else np.ascontiguousarray(init_state, np.float64)
    extra = None
    if getattr(batch, "extra", None):
        names = ("w_noise", "tau_w_e", "cF_ee", "cF_ei", "cF_ie", "cF_ii")
        extra = np.empty((ni, 6))
        for j, name in enumerate(names):
            extra[:, j] = batch.extra[name] if name in batch.extra else getattr(m, name)
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    rc = lib().oracle_run(C.byref(m), C.byref(r), n, np.ascontiguousarray(conn.weights, np.float64),
                          np.ascontiguousarray(conn.tract_mm, np.float64), ni,
                          np.ascontiguousarray(batch.S), np.ascontiguousarray(batch.b_e),
                          np.ascontiguousarray(batch.a_e), np.ascontiguousarray(batch.v), ids,
                          _ptr(init), _ptr(extra), out["final"], _ptr(out["samples"]), _ptr(out["trace"]),
                          _ptr(out["fc"]), _ptr(out["stats"]), out["flags"], int(n_threads))
    if rc != 0:
        raise ValueError("oracle_run rejected its arguments")
    return out
