"""The GPU model arithmetic (adex_model.h, single-precision drift) compiled for
the host and compared with the FP64 oracle, so that rewrites of the model code
are checked on machines without a GPU. The kernels' own parity is the GPU
tests' job; here the bound is what FP32 evaluation of the same quantities
allows. Errors of the jet components are measured against the size of the
terms they enter (F, and the first- and second-order terms of F's Taylor
expansion over the inputs (xe, xi): F_a xe, F_ab xe xi, ...), so that a
derivative passing through zero is measured on the scale it matters at. FP32
evaluation of erfc far in its tail multiplies the input rounding by about
2 Z^2 (Z up to ~5 here): median errors of a few 1e-8, 5e-5 at the 99th
percentile and 2e-4 at worst are the bound.
"""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_13337_amd", "csrc")


class VModel(C.Structure):
    """Mirror of vadx_model (include/vadx.h), filled from the oracle's preset."""
    _fields_ = [(f, C.c_double) for f in (
        "C_m", "g_L", "E_e", "E_i", "Q_e", "Q_i", "tau_e", "tau_i", "K_e", "K_i", "N_e", "N_i", "T",
        "E_L_e", "E_L_i", "tau_w_e", "tau_w_i", "b_i", "a_i", "cF_ee", "cF_ei", "cF_ie", "cF_ii",
        "tau_OU", "sigma_OU", "w_noise", "muV0", "dmuV0", "sV0", "dsV0", "tN0", "dtN0",
        "rate_max", "E_init", "I_init", "x_floor")] + [("P_e", C.c_double * 10),
                                                        ("P_i", C.c_double * 10)]


def vmodel(om):
    v = VModel()
    for name, _ in VModel._fields_:
        if name in ("P_e", "P_i"):
            getattr(v, name)[:] = list(getattr(om, name))
        else:
            setattr(v, name, getattr(om, name))
    return v


@pytest.fixture(scope="module")
def mh(tmp_path_factory):
    out = tmp_path_factory.mktemp("model_host") / "libmodel_host.so"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-ffp-contract=off",
                           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                           os.path.join(ROOT, "tests", "helpers", "model_host.cpp"),
                           "-o", str(out)])
    L = C.CDLL(str(out))
    f32 = np.ctypeslib.ndpointer(np.float32, flags="C")
    f64 = np.ctypeslib.ndpointer(np.float64, flags="C")
    L.mh_tf.argtypes = [C.POINTER(VModel), C.c_int, C.c_float, C.c_float, C.c_float, f32]
    L.mh_drift.argtypes = [C.POINTER(VModel), f32, C.c_float, C.c_float, C.c_float, f32]
    L.mh_step.argtypes = [C.POINTER(VModel), C.c_int, C.c_double, f64, C.c_float, C.c_float,
                          C.c_float, C.c_double]
    L.mh_step.restype = C.c_int
    return L


@pytest.mark.parametrize("preset", ["literature-B", "paper-T1"])
@pytest.mark.parametrize("tau_i", [None, 3.0])
def test_transfer_jets_against_oracle(mh, preset, tau_i):
    over = {} if tau_i is None else {"tau_i": tau_i}
    om = oracle.model(preset, **over)
    vm = vmodel(om)
    rng = np.random.default_rng(7)
    rel = []
    for t in range(3000):
        xe, xi = (float(np.float32(10 ** u)) for u in rng.uniform(-5, -0.5, 2))
        W = float(np.float32(rng.uniform(-50, 500)))
        pop = t % 2
        o = oracle.tf(om, pop, xe, xi, W)
        if o[0] < 1e-9:          # rates below 1e-6 Hz carry no information in FP32
            continue
        g = np.zeros(7, np.float32)
        mh.mh_tf(C.byref(vm), pop, xe, xi, W, g)
        assert abs(g[6] - o[6]) <= 1e-5 * abs(o[6]) + 1e-4          # mu_V (mV)
        s1 = o[0] + abs(o[1]) * xe + abs(o[2]) * xi
        s2 = o[0] + abs(o[3]) * xe * xe + abs(o[4]) * xe * xi + abs(o[5]) * xi * xi
        w = np.array([1 / o[0], xe / s1, xi / s1, xe * xe / s2, xe * xi / s2, xi * xi / s2])
        rel.append(np.abs(g[:6] - o[:6]) * w)
    rel = np.array(rel)
    assert len(rel) > 1000
    assert np.all(np.median(rel, 0) < 1e-6), np.median(rel, 0)
    assert np.all(np.quantile(rel, 0.99, axis=0) < 5e-5), np.quantile(rel, 0.99, axis=0)
    assert np.all(rel.max(0) < 2e-4), rel.max(0)


def test_drift_and_step_against_oracle(mh):
    om = oracle.model("literature-B")
    vm = vmodel(om)
    rng = np.random.default_rng(3)
    for t in range(300):
        E, I = rng.uniform(1e-4, 0.05, 2)
        X = np.array([E, I, rng.uniform(0, 1e-4) * E, 0.0, rng.uniform(0, 1e-4) * I,
                      rng.uniform(0, 200), 0.0, rng.normal(0, 1e-3)])
        X[3] = rng.uniform(-0.5, 0.5) * np.sqrt(X[2] * X[4])
        X = X.astype(np.float32).astype(np.float64)
        c, be, ae = (float(np.float32(v)) for v in (rng.uniform(0, 0.02), rng.uniform(0, 120),
                                                    rng.uniform(0, 8)))
        o = oracle.drift(om, X, c, be, ae)
        g = np.zeros(8, np.float32)
        mh.mh_drift(C.byref(vm), X.astype(np.float32), c, be, ae, g)
        scale = np.abs(o) + np.abs(X) / 20.0 + 1e-12       # drift against state / T
        # eq. (2) sums terms of size |C| |grad F| / T that can cancel: the
        # single-precision rounding is relative to those terms
        xo = X[0] + c + om.w_noise * X[7]
        grads = 0.0
        for pop, xe, xi, W in ((0, xo + om.cF_ee, X[1] + om.cF_ei, X[5]),
                               (1, xo + om.cF_ie, X[1] + om.cF_ii, X[6])):
            t = oracle.tf(om, pop, max(xe, om.x_floor), max(xi, om.x_floor), W)
            grads += abs(t[1]) + abs(t[2])
        scale[2:5] += 2.0 * (abs(X[2]) + abs(X[3]) + abs(X[4])) * grads / om.T
        assert np.all(np.abs(g - o) <= 1e-4 * scale), (X, g, o)
        # one Heun step (drift in FP32, state in FP64) against the FP64 step
        Xg = X.copy()
        mh.mh_step(C.byref(vm), 0, 0.1, Xg, c, be, ae, 1e-5)
        Xo, _ = oracle.step_region(om, X, c, be, ae, 1e-5 / (om.sigma_OU / om.tau_OU * np.sqrt(0.1)))
        # the increment dt (f0 + f1) / 2 carries the drifts' error bound above
        assert np.all(np.abs(Xg - Xo) <= 1e-5 * (np.abs(Xo) + np.abs(X)) + 0.1 * 1e-4 * scale + 1e-15), \
            (Xg, Xo)


def _host_trajectory(mh, om, conn, batch, i, n_steps, seed=0):
    """Free-running network of the single-precision model code on the host:
    FP32 drift, FP64 state, coupling summed in FP32 from the FP32 rate
    history (as the kernel's ring holds it), the oracle's Philox normals.
    Returns the trace [steps, 8, n] rounded to FP32 as the kernel records it."""
    vm = vmodel(om)
    n = conn.n
    W = oracle.normalise_rows(conn.weights).astype(np.float32)
    d = oracle.delays(conn.tract_mm, batch.v[i], 0.1)
    rows = [np.nonzero(W[k])[0] for k in range(n)]
    X = np.zeros((n, 8))
    X[:, 0], X[:, 1] = om.E_init, om.I_init
    H = np.zeros((n_steps + 1, n), np.float32)
    H[0] = np.float32(om.E_init)
    tr = np.zeros((n_steps, 8, n))
    gsc = om.sigma_OU / om.tau_OU * np.sqrt(0.1)
    S = np.float32(batch.S[i])
    for s in range(n_steps):
        for k in range(n):
            acc = np.float32(0.0)
            for j in rows[k]:
                acc = np.float32(acc + W[k, j] * H[max(s - d[k, j], 0), j])
            x = np.ascontiguousarray(X[k])
            mh.mh_step(C.byref(vm), 0, 0.1, x, S * acc, float(batch.b_e[i]), float(batch.a_e[i]),
                       gsc * oracle.normal(seed, i, s, k))
            X[k] = x
        H[s + 1] = X[:, 0].astype(np.float32)
        tr[s] = X.T.astype(np.float32)
    return tr


def test_anchored_check_on_single_precision_trajectories(mh):
    """The re-anchored step check of the GPU parity tests, run on free
    trajectories of the host build of the same single-precision model code:
    it passes for a weakly and a strongly coupled network (the latter with
    steps whose conditioning the check has to account for), and it fails when
    the oracle's model differs by 1 % in one constant (T)."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from parity_checks import anchored_check

    from paper_2311_13337_amd import inputs
    conn = inputs.synthetic_connectome(68)
    batch = inputs.grid_small()
    cfg = inputs.RunConfig(n_steps=300, transient_steps=0, n_trace_steps=300)
    om = oracle.model("literature-B")
    for i in (0, 6):
        tr = _host_trajectory(mh, om, conn, batch, i, 300)
        err, _ = anchored_check(oracle, om, cfg, conn, batch, i, tr)
        assert err.max() < 1.0, (i, err.max())
    wrong = oracle.model("literature-B", T=om.T * 1.01)
    tr = _host_trajectory(mh, om, conn, batch, 0, 300)
    err, _ = anchored_check(oracle, wrong, cfg, conn, batch, 0, tr)
    assert err.max() > 1.0
