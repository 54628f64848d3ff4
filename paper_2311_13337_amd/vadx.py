"""ctypes binding of libvadx (include/vadx.h): the same entry points, argument
marshalling only. Device memory (the workspace) and the stream come from
PyTorch; every step of the computation runs in the library's HIP kernels.

Loading fails loudly when the library has not been built: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvadx.so")

VADX_OK, VADX_E_ARG, VADX_E_OOM, VADX_E_HIP, VADX_E_STATE, VADX_E_NUMERIC, VADX_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
VADX_HOST, VADX_DEVICE = 0, 1
VADX_PRESET_LITERATURE_B, VADX_PRESET_PAPER_T1 = 0, 1
VADX_HEUN, VADX_EULER = 0, 1
PRESETS = {"literature-B": VADX_PRESET_LITERATURE_B, "paper-T1": VADX_PRESET_PAPER_T1}
STAT_NAMES = ("fc_mean", "fc_std", "fc_sc_corr", "rate_mean_hz", "rate_std_hz", "sync_index")

EXPORTS = ("vadx_create", "vadx_destroy", "vadx_last_error", "vadx_model_defaults",
           "vadx_set_model", "vadx_add_connectome", "vadx_set_batch", "vadx_set_trace",
           "vadx_plan", "vadx_integrate", "vadx_sync", "vadx_read_stats", "vadx_read_fc",
           "vadx_read_samples", "vadx_read_state", "vadx_read_trace", "vadx_instance_shape",
           "vadx_enable_timing", "vadx_kernel_time", "vadx_region_step_ops",
           "vadx_set_launch", "vadx_set_noise_keys", "vadx_set_graph", "vadx_autotune", "vadx_set_waves_per_simd", "vadx_launch_info", "vadx_class_lanes", "vadx_wave_slack", "vadx_mlp_create", "vadx_mlp_destroy", "vadx_mlp_last_error",
           "vadx_mlp_fit_target_norm", "vadx_mlp_get_target_norm", "vadx_mlp_set_target_norm",
           "vadx_mlp_get_params", "vadx_mlp_set_params", "vadx_mlp_grad", "vadx_mlp_train",
           "vadx_mlp_predict", "vadx_mlp_select", "vadx_analysis_defaults",
           "vadx_analysis_ws_bytes", "vadx_analyze_series", "vadx_analyze",
           "vadx_analysis_kernel_time", "vadx_set_reference_fc", "vadx_top_k", "vadx_top_k_noalloc",
           "vadx_set_instance_param", "vadx_bold_defaults", "vadx_bold_series", "vadx_bold")
INSTANCE_PARAMS = {"w_noise": 0, "tau_w_e": 1, "cF_ee": 2, "cF_ei": 3, "cF_ie": 4, "cF_ii": 5}
ANALYSIS_KERNELS = ("an_transpose_kernel", "an_welch_kernel", "an_hilbert_kernel", "an_pli_kernel",
                    "an_ud_kernel", "an_final_kernel")
ANALYSIS_NAMES = ("psd_fmax_hz", "psd_ampmax", "psd_slope_a", "psd_log10_b", "mean_pli",
                  "ud_up_ms", "ud_down_ms")
MLP_PARAMS = 17926


class VadxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"vadx status {status}: {msg}")
        self.status = status


class vadx_model(C.Structure):
    _fields_ = [(f, C.c_double) for f in (
        "C_m", "g_L", "E_e", "E_i", "Q_e", "Q_i", "tau_e", "tau_i", "K_e", "K_i", "N_e", "N_i",
        "T", "E_L_e", "E_L_i", "tau_w_e", "tau_w_i", "b_i", "a_i", "cF_ee", "cF_ei", "cF_ie",
        "cF_ii", "tau_OU", "sigma_OU", "w_noise", "muV0", "dmuV0", "sV0", "dsV0", "tN0", "dtN0",
        "rate_max", "E_init", "I_init", "x_floor")] + [
        ("P_e", C.c_double * 10), ("P_i", C.c_double * 10)]


class vadx_run(C.Structure):
    _fields_ = [("dt_ms", C.c_double), ("n_steps", C.c_int64), ("transient_steps", C.c_int64),
                ("tavg_steps", C.c_int64), ("n_trace_steps", C.c_int64), ("seed", C.c_uint32),
                ("integrator", C.c_int32), ("noise_off", C.c_int32), ("chunk_steps", C.c_int32),
                ("fc_min_std", C.c_double)]


class vadx_mlp_cfg(C.Structure):
    _fields_ = [("x_lo", C.c_float * 4), ("x_hi", C.c_float * 4), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("hip_stream", C.c_void_p)]


class vadx_analysis_cfg(C.Structure):
    _fields_ = [("window", C.c_int32), ("segment", C.c_int32), ("fit_lo_hz", C.c_double),
                ("fit_hi_hz", C.c_double), ("ud_band", C.c_float), ("ud_min_range_khz", C.c_float)]


class vadx_analysis(C.Structure):
    _fields_ = [(f, C.c_float) for f in ANALYSIS_NAMES] + [
        ("reserved", C.c_float), ("psd_peak_bin", C.c_int32), ("psd_fit_bins", C.c_int32),
        ("ud_up_count", C.c_int32), ("ud_down_count", C.c_int32),
        ("ud_up_samples", C.c_int64), ("ud_down_samples", C.c_int64)]


class vadx_bold_cfg(C.Structure):
    _fields_ = [(f, C.c_double) for f in ("kappa", "gamma", "tau0", "alpha", "E0", "V0", "k1",
                                          "k2", "k3", "tr_ms")]


class vadx_stats(C.Structure):
    _fields_ = [(f, C.c_float) for f in STAT_NAMES] + [("flags", C.c_uint32),
                                                        ("fc_fit", C.c_float)]


_lib = None


def lib():
    """Loads libvadx.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                               "(python -m paper_2311_13337_amd.build)")
        # The library and PyTorch must share one HIP runtime (the stream and
        # workspace come from PyTorch): load PyTorch's runtime first so the
        # library's libamdhip64 dependency resolves to it.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P, vp = C.POINTER, C.c_void_p
        st = C.c_int32
        sig = {
            "vadx_create": (st, [C.c_int, vp, P(vp)]),
            "vadx_destroy": (None, [vp]),
            "vadx_last_error": (C.c_char_p, [vp]),
            "vadx_model_defaults": (st, [C.c_int, P(vadx_model)]),
            "vadx_set_model": (st, [vp, P(vadx_model)]),
            "vadx_add_connectome": (st, [vp, C.c_int32, vp, vp, P(C.c_int32)]),
            "vadx_set_batch": (st, [vp, C.c_int64, vp, vp, vp, vp, vp]),
            "vadx_set_trace": (st, [vp, C.c_int64, vp]),
            "vadx_set_noise_keys": (st, [vp, C.c_int64, vp]),
            "vadx_set_graph": (st, [vp, C.c_int32]),
            "vadx_autotune": (st, [vp, P(vadx_run), vp, C.c_size_t, C.c_char_p, C.c_int32,
                                   P(C.c_int32), P(C.c_int32), P(C.c_int32)]),
            "vadx_set_waves_per_simd": (st, [vp, C.c_int32]),
            "vadx_launch_info": (st, [vp, P(C.c_int32), P(C.c_int32), P(C.c_int32), P(C.c_int32)]),
            "vadx_class_lanes": (st, [vp, C.c_int32, C.c_int32, P(C.c_int32)]),
            "vadx_wave_slack": (st, [vp, C.c_int32, P(C.c_int32)]),
            "vadx_plan": (st, [vp, P(vadx_run), P(C.c_size_t)]),
            "vadx_integrate": (st, [vp, P(vadx_run), vp, C.c_size_t]),
            "vadx_sync": (st, [vp]),
            "vadx_read_stats": (st, [vp, C.c_int64, C.c_int64, vp, C.c_int32]),
            "vadx_read_fc": (st, [vp, C.c_int64, vp, C.c_int32]),
            "vadx_read_samples": (st, [vp, C.c_int64, vp, C.c_int32]),
            "vadx_read_state": (st, [vp, C.c_int64, vp, C.c_int32]),
            "vadx_read_trace": (st, [vp, C.c_int64, vp, C.c_int32]),
            "vadx_instance_shape": (st, [vp, C.c_int64, P(C.c_int32), P(C.c_int64)]),
            "vadx_enable_timing": (st, [vp, C.c_int32]),
            "vadx_set_launch": (st, [vp, C.c_int32, C.c_int32, C.c_int32]),
            "vadx_kernel_time": (st, [vp, P(C.c_int64), P(C.c_double), P(C.c_int64),
                                      P(C.c_double)]),
            "vadx_region_step_ops": (st, [C.c_int32, P(C.c_double), P(C.c_double),
                                          P(C.c_double)]),
            "vadx_mlp_create": (st, [vp, P(vadx_mlp_cfg), vp, P(vp)]),
            "vadx_mlp_destroy": (None, [vp]),
            "vadx_mlp_last_error": (C.c_char_p, [vp]),
            "vadx_mlp_fit_target_norm": (st, [vp, vp, C.c_int64]),
            "vadx_mlp_get_target_norm": (st, [vp, vp, vp]),
            "vadx_mlp_set_target_norm": (st, [vp, vp, vp]),
            "vadx_mlp_get_params": (st, [vp, vp]),
            "vadx_mlp_set_params": (st, [vp, vp]),
            "vadx_mlp_grad": (st, [vp, vp, vp, C.c_int64, vp, P(C.c_float)]),
            "vadx_mlp_train": (st, [vp, vp, vp, C.c_int64, C.c_int32, C.c_int32, vp]),
            "vadx_mlp_predict": (st, [vp, vp, C.c_int64, vp, vp, vp, C.c_int32, C.c_int32]),
            "vadx_mlp_select": (st, [vp, vp, C.c_int64, C.c_int64, C.c_float, C.c_uint32, vp, vp,
                                     C.c_int64, P(C.c_int64)]),
            "vadx_analysis_defaults": (st, [P(vadx_analysis_cfg)]),
            "vadx_analysis_ws_bytes": (st, [C.c_int64, C.c_int32, C.c_int64, P(vadx_analysis_cfg),
                                            P(C.c_size_t)]),
            "vadx_analyze_series": (st, [vp, vp, C.c_int64, C.c_int32, C.c_int64, C.c_double,
                                         P(vadx_analysis_cfg), vp, C.c_size_t, vp, vp, vp]),
            "vadx_analyze": (st, [vp, P(vadx_analysis_cfg), vp, C.c_size_t, vp]),
            "vadx_analysis_kernel_time": (st, [vp, vp, vp]),
            "vadx_set_reference_fc": (st, [vp, C.c_int32, vp]),
            "vadx_top_k": (st, [vp, vp, C.c_int64, C.c_int32, vp, vp]),
            "vadx_top_k_noalloc": (st, [vp, vp, C.c_int64, C.c_int32, vp, vp]),
            "vadx_set_instance_param": (st, [vp, C.c_int32, C.c_int64, vp]),
            "vadx_bold_defaults": (st, [P(vadx_bold_cfg)]),
            "vadx_bold_series": (st, [vp, vp, C.c_int64, C.c_int32, C.c_int64, C.c_double,
                                      P(vadx_bold_cfg), vp, P(C.c_int32)]),
            "vadx_bold": (st, [vp, P(vadx_bold_cfg), vp, P(C.c_int32)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def vadx_region_step_ops(integrator: int = VADX_HEUN):
    """(fp32 FLOPs, fp64 FLOPs, transcendentals) of one region-step, coupling excluded."""
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    s = lib().vadx_region_step_ops(integrator, C.byref(a), C.byref(b), C.byref(c))
    if s != VADX_OK:
        raise VadxError(s, "bad integrator")
    return a.value, b.value, c.value


def vadx_model_defaults(preset: int = VADX_PRESET_LITERATURE_B) -> vadx_model:
    m = vadx_model()
    s = lib().vadx_model_defaults(preset, C.byref(m))
    if s != VADX_OK:
        raise VadxError(s, "bad preset")
    return m


class Context:
    """One vadx_ctx bound to a device and a HIP stream (default: torch's
    current stream on that device). Methods are the ABI calls."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        self._check(lib().vadx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h
        self.device = device

    def _check(self, s: int):
        if s != VADX_OK:
            msg = lib().vadx_last_error(getattr(self, "h", None))
            raise VadxError(s, (msg or b"").decode())

    def close(self):
        if getattr(self, "h", None):
            lib().vadx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def vadx_set_model(self, m: vadx_model):
        self._check(lib().vadx_set_model(self.h, C.byref(m)))

    def vadx_add_connectome(self, weights: np.ndarray, tract_mm: np.ndarray) -> int:
        w = np.ascontiguousarray(weights, np.float64)
        L = np.ascontiguousarray(tract_mm, np.float64)
        cid = C.c_int32()
        self._check(lib().vadx_add_connectome(self.h, w.shape[0], _ptr(w), _ptr(L), C.byref(cid)))
        return cid.value

    def vadx_set_batch(self, S, b_e, a_e, v, conn=None):
        arrs = [np.ascontiguousarray(x, np.float32) for x in (S, b_e, a_e, v)]
        cp = None if conn is None else np.ascontiguousarray(conn, np.int32)
        self._keep = (arrs, cp)
        self._check(lib().vadx_set_batch(self.h, arrs[0].shape[0], *[_ptr(x) for x in arrs],
                                         None if cp is None else _ptr(cp)))

    def vadx_autotune(self, run, ws_ptr, ws_bytes, cache_path=None, trial_steps=0):
        lanes, items, waves = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(lib().vadx_autotune(self.h, C.byref(run), C.c_void_p(ws_ptr), ws_bytes,
                                        cache_path.encode() if cache_path else None, trial_steps,
                                        C.byref(lanes), C.byref(items), C.byref(waves)))
        return lanes.value, items.value, waves.value

    def vadx_launch_info(self):
        g, t, gr, b = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        self._check(lib().vadx_launch_info(self.h, C.byref(g), C.byref(t), C.byref(gr), C.byref(b)))
        return {"groups": g.value, "block_threads": t.value, "grid": gr.value,
                "steps_per_block": b.value}

    def vadx_class_lanes(self, n_regions: int, lanes: int = -1) -> int:
        """Sets (lanes > 0), clears (0) or only reads (-1) the lane budget of
        instances with n_regions regions; returns the budget in effect."""
        cur = C.c_int32()
        self._check(lib().vadx_class_lanes(self.h, n_regions, lanes, C.byref(cur)))
        return cur.value

    def vadx_set_waves_per_simd(self, waves: int):
        self._check(lib().vadx_set_waves_per_simd(self.h, waves))

    def vadx_wave_slack(self, slack: int = -1) -> int:
        """Sets the wave slack (0 or 1; -1 leaves it) and returns the setting."""
        cur = C.c_int32(0)
        self._check(lib().vadx_wave_slack(self.h, slack, C.byref(cur)))
        return cur.value

    def vadx_set_graph(self, on: bool):
        self._check(lib().vadx_set_graph(self.h, 1 if on else 0))

    def vadx_set_noise_keys(self, keys):
        a = np.ascontiguousarray(keys, np.uint32)
        self._check(lib().vadx_set_noise_keys(self.h, a.shape[0], _ptr(a) if a.size else None))

    def vadx_set_instance_param(self, name: str, values=None):
        p = INSTANCE_PARAMS[name]
        if values is None:
            n = len(self._keep[0][0])
            self._check(lib().vadx_set_instance_param(self.h, p, n, None))
            return
        a = np.ascontiguousarray(values, np.float64)
        self._check(lib().vadx_set_instance_param(self.h, p, a.shape[0], _ptr(a)))

    def vadx_set_trace(self, inst):
        a = np.ascontiguousarray(inst, np.int64)
        self._check(lib().vadx_set_trace(self.h, a.shape[0], _ptr(a) if a.size else None))

    def vadx_plan(self, run: vadx_run) -> int:
        b = C.c_size_t()
        self._check(lib().vadx_plan(self.h, C.byref(run), C.byref(b)))
        return b.value

    def vadx_integrate(self, run: vadx_run, ws_ptr: int, ws_bytes: int):
        self._check(lib().vadx_integrate(self.h, C.byref(run), C.c_void_p(ws_ptr), ws_bytes))

    def vadx_sync(self):
        self._check(lib().vadx_sync(self.h))

    def vadx_instance_shape(self, inst: int):
        n, ns = C.c_int32(), C.c_int64()
        self._check(lib().vadx_instance_shape(self.h, inst, C.byref(n), C.byref(ns)))
        return n.value, ns.value

    def vadx_read_stats(self, first: int, count: int) -> np.ndarray:
        out = (vadx_stats * count)()
        self._check(lib().vadx_read_stats(self.h, first, count, C.cast(out, C.c_void_p), VADX_HOST))
        arr = np.ctypeslib.as_array(out).copy()
        return arr

    def _read(self, fn, inst, shape):
        out = np.zeros(shape, np.float32)
        self._check(getattr(lib(), fn)(self.h, inst, _ptr(out), VADX_HOST))
        return out

    def vadx_read_fc(self, inst: int) -> np.ndarray:
        n, _ = self.vadx_instance_shape(inst)
        return self._read("vadx_read_fc", inst, (n, n))

    def vadx_read_samples(self, inst: int) -> np.ndarray:
        n, ns = self.vadx_instance_shape(inst)
        return self._read("vadx_read_samples", inst, (ns, n))

    def vadx_read_state(self, inst: int) -> np.ndarray:
        n, _ = self.vadx_instance_shape(inst)
        out = np.zeros((8, n), np.float64)
        self._check(lib().vadx_read_state(self.h, inst, _ptr(out), VADX_HOST))
        return out

    def vadx_read_trace(self, slot: int, inst: int, n_trace_steps: int) -> np.ndarray:
        n, _ = self.vadx_instance_shape(inst)
        return self._read("vadx_read_trace", slot, (n_trace_steps, 8, n))

    def vadx_set_launch(self, mode: int = 0, wg_instances: int = 0, item_steps: int = 0):
        self._check(lib().vadx_set_launch(self.h, mode, wg_instances, item_steps))

    def vadx_enable_timing(self, on: bool = True):
        self._check(lib().vadx_enable_timing(self.h, 1 if on else 0))

    def vadx_kernel_time(self):
        a, b, c, d = C.c_int64(), C.c_double(), C.c_int64(), C.c_double()
        self._check(lib().vadx_kernel_time(self.h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return a.value, b.value, c.value, d.value

    def vadx_analyze_series(self, samples, n_samples: int, n: int, period_ms: float,
                            cfg: "vadx_analysis_cfg", ws, out, psd_out=None, pli_out=None):
        """samples: device tensor [n_inst][n_samples][n] float32; ws: device tensor
        (uint8, 256-byte aligned); out: device tensor of n_inst * 64 bytes."""
        n_inst = samples.shape[0]
        self._check(lib().vadx_analyze_series(
            self.h, C.c_void_p(samples.data_ptr()), n_inst, n, n_samples, period_ms, C.byref(cfg),
            C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(), C.c_void_p(out.data_ptr()),
            None if psd_out is None else C.c_void_p(psd_out.data_ptr()),
            None if pli_out is None else C.c_void_p(pli_out.data_ptr())))

    def vadx_set_reference_fc(self, conn_id: int, fc=None):
        if fc is None:
            self._check(lib().vadx_set_reference_fc(self.h, conn_id, None))
            return
        a = np.ascontiguousarray(fc, np.float32)
        self._check(lib().vadx_set_reference_fc(self.h, conn_id, _ptr(a)))

    def vadx_top_k(self, score, k: int):
        """score: device float32 tensor; returns (indices, scores) as device tensors."""
        import torch
        idx = torch.empty(max(k, 1), dtype=torch.int64, device=score.device)
        val = torch.empty(max(k, 1), dtype=torch.float32, device=score.device)
        self._check(lib().vadx_top_k(self.h, C.c_void_p(score.data_ptr()), score.numel(), k,
                                     C.c_void_p(idx.data_ptr()), C.c_void_p(val.data_ptr())))
        return idx[:k], val[:k]

    def vadx_top_k_noalloc(self, score, k: int, idx, val=None):
        """As vadx_top_k into caller-given device tensors idx (int64, >= k) and
        val (float32, nullable); the library allocates nothing."""
        self._check(lib().vadx_top_k_noalloc(self.h, C.c_void_p(score.data_ptr()), score.numel(), k,
                                             C.c_void_p(idx.data_ptr()),
                                             C.c_void_p(val.data_ptr()) if val is not None else None))

    def vadx_bold_series(self, samples, n_samples: int, n: int, period_ms: float,
                         cfg: "vadx_bold_cfg" = None):
        """samples: device tensor [n_inst][n_samples][n]; returns the device
        tensor [n_inst][n_tr][n] of BOLD samples."""
        import torch
        cfg = cfg or vadx_bold_defaults()
        n_inst = samples.shape[0]
        n_tr = int(np.floor(n_samples * period_ms / cfg.tr_ms + 1e-9))
        out = torch.empty((n_inst, max(n_tr, 0), n), dtype=torch.float32, device=samples.device)
        got = C.c_int32()
        self._check(lib().vadx_bold_series(self.h, C.c_void_p(samples.data_ptr()), n_inst, n,
                                           n_samples, period_ms, C.byref(cfg),
                                           C.c_void_p(out.data_ptr()), C.byref(got)))
        assert got.value == n_tr
        return out

    def vadx_bold(self, cfg: "vadx_bold_cfg", out):
        got = C.c_int32()
        self._check(lib().vadx_bold(self.h, C.byref(cfg), C.c_void_p(out.data_ptr()),
                                    C.byref(got)))
        return got.value

    def vadx_analyze(self, cfg: "vadx_analysis_cfg", ws, out):
        self._check(lib().vadx_analyze(self.h, C.byref(cfg), C.c_void_p(ws.data_ptr()),
                                       ws.numel() * ws.element_size(), C.c_void_p(out.data_ptr())))


def analysis_kernel_time(ctx: "Context"):
    """{kernel: (launches, ms)} of the analysis launches since the last call."""
    n = np.zeros(6, np.int64)
    ms = np.zeros(6, np.float64)
    ctx._check(lib().vadx_analysis_kernel_time(ctx.h, _ptr(n), _ptr(ms)))
    return {k: (int(a), float(b)) for k, a, b in zip(ANALYSIS_KERNELS, n, ms)}


def vadx_bold_defaults() -> vadx_bold_cfg:
    c = vadx_bold_cfg()
    s = lib().vadx_bold_defaults(C.byref(c))
    if s != VADX_OK:
        raise VadxError(s, "BOLD defaults")
    return c


def vadx_analysis_defaults() -> vadx_analysis_cfg:
    c = vadx_analysis_cfg()
    s = lib().vadx_analysis_defaults(C.byref(c))
    if s != VADX_OK:
        raise VadxError(s, "analysis defaults")
    return c


def vadx_analysis_ws_bytes(n_samples: int, n_max: int, regions_per_pass: int,
                           cfg: vadx_analysis_cfg | None = None) -> int:
    cfg = cfg or vadx_analysis_defaults()
    b = C.c_size_t()
    s = lib().vadx_analysis_ws_bytes(n_samples, n_max, regions_per_pass, C.byref(cfg), C.byref(b))
    if s != VADX_OK:
        raise VadxError(s, "invalid analysis sizes or settings")
    return b.value


def analysis_to_numpy(out) -> np.ndarray:
    """Device tensor of vadx_analysis records -> numpy structured array."""
    raw = out.cpu().numpy().tobytes()
    n = len(raw) // C.sizeof(vadx_analysis)
    arr = (vadx_analysis * n).from_buffer_copy(raw)
    return np.ctypeslib.as_array(arr).copy()


def analysis_out(n_inst: int, device: int = 0):
    """Device buffer for n_inst vadx_analysis records."""
    import torch
    return torch.zeros(n_inst * C.sizeof(vadx_analysis), dtype=torch.uint8, device=f"cuda:{device}")


def make_run(cfg, integrator: int = VADX_HEUN, noise_off: bool = False, chunk_steps: int = 0,
             n_trace_steps=None) -> vadx_run:
    """vadx_run from an object with dt_ms, n_steps, transient_steps, tavg_steps, seed."""
    return vadx_run(dt_ms=cfg.dt_ms, n_steps=cfg.n_steps, transient_steps=cfg.transient_steps,
                    tavg_steps=cfg.tavg_steps,
                    n_trace_steps=cfg.n_trace_steps if n_trace_steps is None else n_trace_steps,
                    seed=cfg.seed, integrator=integrator, noise_off=1 if noise_off else 0,
                    chunk_steps=chunk_steps, fc_min_std=getattr(cfg, "fc_min_std", 1e-9))


class Sweep:
    """Convenience driver: one context, connectomes, a batch, a planned run and
    a torch-allocated workspace."""

    def __init__(self, device: int = 0, model: vadx_model | None = None, stream=None):
        import torch
        self.torch = torch
        self.ctx = Context(device, stream)
        self.device = device
        if model is not None:
            self.ctx.vadx_set_model(model)
        self.ws = None
        self.run = None

    def add_connectome(self, conn) -> int:
        return self.ctx.vadx_add_connectome(conn.weights, conn.tract_mm)

    def set_batch(self, batch, conn_ids=None, noise_keys=None):
        conn = batch.conn if conn_ids is None else np.asarray(conn_ids)[batch.conn]
        self.ctx.vadx_set_batch(batch.S, batch.b_e, batch.a_e, batch.v, conn)
        if noise_keys is not None:
            self.ctx.vadx_set_noise_keys(noise_keys)
        for name, values in (getattr(batch, "extra", None) or {}).items():
            self.ctx.vadx_set_instance_param(name, values)

    def plan(self, run: vadx_run, trace=()):
        self.ctx.vadx_set_trace(list(trace))
        nbytes = self.ctx.vadx_plan(run)
        if self.ws is None or self.ws.numel() < nbytes + 256:
            self.ws = None
            self.ws = self.torch.empty(nbytes + 256, dtype=self.torch.uint8,
                                       device=f"cuda:{self.device}")
        self.run = run
        self.nbytes = nbytes
        return nbytes

    def autotune(self, cache_path=None, trial_steps=0):
        """Tunes the launch shape for the planned run, then re-plans. The
        workspace is first grown to what the run needs with wave slack (its
        rings can be deeper), so that the trials can include it."""
        slack = self.ctx.vadx_wave_slack()
        self.ctx.vadx_wave_slack(1)
        self.plan(self.run)
        self.ctx.vadx_wave_slack(slack)
        self.plan(self.run)
        choice = self.ctx.vadx_autotune(self.run, self.ws_ptr(), self.ws.numel() - 256, cache_path,
                                        trial_steps)
        self.plan(self.run)
        return choice

    def ws_ptr(self):
        p = self.ws.data_ptr()
        return (p + 255) // 256 * 256

    def integrate(self):
        self.ctx.vadx_integrate(self.run, self.ws_ptr(), self.nbytes)

    def sync(self):
        self.ctx.vadx_sync()

    def stats(self, first: int = 0, count: int | None = None) -> np.ndarray:
        if count is None:
            count = self.n_inst
        s = self.ctx.vadx_read_stats(first, count)
        return s

    @property
    def n_inst(self):
        return len(self.ctx._keep[0][0])


class Mlp:
    """The surrogate network (vadx_mlp_*). Device data are torch CUDA float32
    tensors; their pointers are passed through unchanged."""

    def __init__(self, init_params, x_lo, x_hi, lr=1e-3, betas=(0.9, 0.999), eps=1e-8,
                 stream=None, device: int = 0):
        import torch
        self.torch = torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        cfg = vadx_mlp_cfg()
        cfg.x_lo[:] = [float(v) for v in x_lo]
        cfg.x_hi[:] = [float(v) for v in x_hi]
        cfg.lr, cfg.beta1, cfg.beta2, cfg.eps = lr, betas[0], betas[1], eps
        cfg.hip_stream = C.c_void_p(stream.cuda_stream)
        p = np.ascontiguousarray(init_params, np.float32)
        assert p.size == MLP_PARAMS
        h = C.c_void_p()
        s = lib().vadx_mlp_create(None, C.byref(cfg), _ptr(p), C.byref(h))
        if s != VADX_OK:
            raise VadxError(s, "vadx_mlp_create")
        self.h = h

    def _check(self, s):
        if s != VADX_OK:
            raise VadxError(s, (lib().vadx_mlp_last_error(self.h) or b"").decode())

    def close(self):
        if getattr(self, "h", None):
            lib().vadx_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _dptr(t, cols):
        assert t.is_cuda and t.dtype.is_floating_point and t.is_contiguous() and t.shape[-1] == cols
        return C.c_void_p(t.data_ptr())

    def fit_target_norm(self, Y):
        self._check(lib().vadx_mlp_fit_target_norm(self.h, self._dptr(Y, 6), Y.shape[0]))

    def target_norm(self):
        m, sd = np.zeros(6, np.float32), np.zeros(6, np.float32)
        self._check(lib().vadx_mlp_get_target_norm(self.h, _ptr(m), _ptr(sd)))
        return m, sd

    def set_target_norm(self, mean, std):
        m = np.ascontiguousarray(mean, np.float32)
        sd = np.ascontiguousarray(std, np.float32)
        self._check(lib().vadx_mlp_set_target_norm(self.h, _ptr(m), _ptr(sd)))

    def params(self):
        out = np.zeros(MLP_PARAMS, np.float32)
        self._check(lib().vadx_mlp_get_params(self.h, _ptr(out)))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        self._check(lib().vadx_mlp_set_params(self.h, _ptr(p)))

    def grad(self, X, Y):
        g = np.zeros(MLP_PARAMS, np.float32)
        loss = C.c_float()
        self._check(lib().vadx_mlp_grad(self.h, self._dptr(X, 4), self._dptr(Y, 6), X.shape[0],
                                        _ptr(g), C.byref(loss)))
        return loss.value, g

    def train(self, X, Y, epochs, batch):
        hist = np.zeros(max(epochs, 1), np.float32)
        self._check(lib().vadx_mlp_train(self.h, self._dptr(X, 4), self._dptr(Y, 6), X.shape[0],
                                         epochs, batch, _ptr(hist)))
        return hist[:epochs]

    def predict(self, X, jacobian=False, score_outputs=None):
        torch = self.torch
        n = X.shape[0]
        Y = torch.empty((n, 6), dtype=torch.float32, device=X.device)
        J = torch.empty((n, 6, 4), dtype=torch.float32, device=X.device) if jacobian else None
        sc = torch.empty(n, dtype=torch.float32, device=X.device) if score_outputs else None
        o0, o1 = score_outputs if score_outputs else (0, 5)
        self._check(lib().vadx_mlp_predict(
            self.h, self._dptr(X, 4), n, C.c_void_p(Y.data_ptr()),
            C.c_void_p(J.data_ptr()) if J is not None else None,
            C.c_void_p(sc.data_ptr()) if sc is not None else None, o0, o1))
        return Y, J, sc

    def select(self, score, k, audit_frac, seed, sel, is_audit=None):
        """Indices (into the device int64 tensor sel) of the k largest scores
        plus the audit sample; returns their count."""
        torch = self.torch
        assert score.is_cuda and score.dtype == torch.float32 and score.is_contiguous()
        assert sel.is_cuda and sel.dtype == torch.int64
        assert is_audit is None or (is_audit.dtype == torch.uint8 and is_audit.numel() >= sel.numel())
        n_sel = C.c_int64()
        self._check(lib().vadx_mlp_select(
            self.h, C.c_void_p(score.data_ptr()), score.numel(), int(k), float(audit_frac),
            int(seed) & 0xFFFFFFFF, C.c_void_p(sel.data_ptr()),
            C.c_void_p(is_audit.data_ptr()) if is_audit is not None else None, sel.numel(),
            C.byref(n_sel)))
        return n_sel.value
