"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

States: |gpu - oracle| <= 1e-4 * max(|oracle|, rms of that state variable over
the window), for every state, region and step of the traced window (the FP32
state must track the FP64 state to 1e-4 relative; the rms floor makes the
criterion meaningful where a variable crosses zero). FC: within 0.02 absolute
over long runs. Both sides draw the same Philox normals.
"""
import os

import numpy as np
import pytest

from paper_2311_13337_amd import inputs, vadx

pytestmark = pytest.mark.gpu

TOL_STATE = 1e-4
TOL_FC = 0.02
NTHREADS = min(16, os.cpu_count() or 1)


def scaled_err(g, o):
    """g, o: [steps, 8, n]. Max of |g - o| / max(|o|, rms_var)."""
    rms = np.sqrt((o ** 2).mean(axis=(0, 2), keepdims=True))
    den = np.maximum(np.abs(o), rms)
    den = np.where(den > 0, den, 1.0)
    e = np.abs(g - o) / den
    return float(e.max()), np.unravel_index(int(e.argmax()), e.shape)


def gpu_model(preset, **over):
    m = vadx.vadx_model_defaults(vadx.PRESETS[preset])
    for k, v in over.items():
        setattr(m, k, v)
    return m


def run_gpu(preset, conns, batch, cfg, trace=(), integrator=0, noise_off=False, chunk=0,
            **over):
    sw = vadx.Sweep(0, gpu_model(preset, **over))
    ids = [sw.add_connectome(c) for c in conns]
    sw.set_batch(batch, conn_ids=ids)
    run = vadx.make_run(cfg, integrator=integrator, noise_off=noise_off, chunk_steps=chunk)
    sw.plan(run, trace=trace)
    sw.integrate()
    sw.sync()
    return sw


def run_oracle(oracle, preset, conn, batch, cfg, inst_ids=None, **kw):
    over = {k: v for k, v in kw.items() if k not in ("integrator", "noise_off")}
    m = oracle.model(preset, **over)
    return oracle.run(m, cfg, conn, batch, inst_ids=inst_ids, n_threads=NTHREADS,
                      integrator=kw.get("integrator", 0), noise_off=kw.get("noise_off", False))


@pytest.mark.parametrize("preset", ["literature-B", "paper-T1"])
def test_first_1000_steps_small_grid(oracle, preset):
    conn = inputs.synthetic_connectome(68)
    batch = inputs.grid_small()
    cfg = inputs.RunConfig(n_steps=1000, transient_steps=0, n_trace_steps=1000)
    print(f"[parity] small grid, preset {preset}, 8 instances x 68 regions x 1000 steps", flush=True)
    sw = run_gpu(preset, [conn], batch, cfg, trace=range(8))
    ref = run_oracle(oracle, preset, conn, batch, cfg)
    for i in range(8):
        g = sw.ctx.vadx_read_trace(i, i, 1000).astype(np.float64)
        e, where = scaled_err(g, ref["trace"][i])
        assert e <= TOL_STATE, f"instance {i}: scaled error {e:.3g} at (step, var, region) {where}"


def test_fc_and_stats_small_grid_full_run(oracle):
    conn = inputs.synthetic_connectome(68)
    batch = inputs.grid_small()
    cfg = inputs.RUN_SMALL
    print("[parity] small grid full 10000 steps, FC + stats", flush=True)
    sw = run_gpu("literature-B", [conn], batch, cfg)
    ref = run_oracle(oracle, "literature-B", conn, batch, cfg)
    st = sw.stats()
    for i in range(len(batch)):
        fc = sw.ctx.vadx_read_fc(i)
        d = np.abs(fc - ref["fc"][i]).max()
        assert d <= TOL_FC, f"instance {i}: max |dFC| {d:.3g}"
        smp = sw.ctx.vadx_read_samples(i)
        assert smp.shape == ref["samples"][i].shape
        g = [st[i][k] for k in vadx.STAT_NAMES]
        o = ref["stats"][i]
        assert abs(g[0] - o[0]) <= TOL_FC and abs(g[1] - o[1]) <= TOL_FC
        assert abs(g[2] - o[2]) <= 2 * TOL_FC
        np.testing.assert_allclose(g[3:5], o[3:5], rtol=1e-2)
        assert abs(g[5] - o[5]) <= TOL_FC
        assert (st[i]["flags"] & 1) == (ref["flags"][i] & 1)


def test_ragged_groups_and_short_delays(oracle):
    """37 regions (not a multiple of 64), 11 instances over several workgroups,
    delays of 1-3 steps, so blocks between barriers are 2 steps long."""
    conn = inputs.synthetic_connectome(37, seed=8, density=0.3, len_lo=0.3, len_hi=1.2)
    rng = np.random.default_rng(1)
    batch = inputs._batch(rng.uniform(0, 0.5, 11), rng.uniform(0, 120, 11), rng.uniform(0, 8, 11),
                          rng.uniform(3.9, 4.1, 11))
    cfg = inputs.RunConfig(n_steps=400, transient_steps=100, n_trace_steps=400, seed=3)
    print("[parity] ragged 37-region groups, 1-3 step delays", flush=True)
    sw = run_gpu("literature-B", [conn], batch, cfg, trace=range(11))
    ref = run_oracle(oracle, "literature-B", conn, batch, cfg)
    for i in range(11):
        g = sw.ctx.vadx_read_trace(i, i, 400).astype(np.float64)
        e, where = scaled_err(g, ref["trace"][i])
        assert e <= TOL_STATE, f"instance {i}: {e:.3g} at {where}"
        np.testing.assert_allclose(sw.ctx.vadx_read_samples(i), ref["samples"][i], rtol=1e-4,
                                   atol=1e-9)


def test_mixed_region_counts_one_launch(oracle):
    """68-, 84- and 200-region networks with different speeds in one launch."""
    conns = [inputs.synthetic_connectome(n) for n in (68, 84, 200)]
    b = inputs.grid_uneven(24, seed=5)
    cfg = inputs.RunConfig(n_steps=600, transient_steps=200, n_trace_steps=300, seed=1)
    print("[parity] mixed 68/84/200 regions, 24 instances", flush=True)
    sw = run_gpu("literature-B", conns, b, cfg, trace=range(24))
    for cls in range(3):
        idx = np.nonzero(b.conn == cls)[0]
        sub = b.subset(idx)
        ref = run_oracle(oracle, "literature-B", conns[cls], sub, cfg, inst_ids=idx)
        for q, i in enumerate(idx):
            g = sw.ctx.vadx_read_trace(int(i), int(i), 300).astype(np.float64)
            e, where = scaled_err(g, ref["trace"][q])
            assert e <= TOL_STATE, f"class {cls} instance {i}: {e:.3g} at {where}"
            fin = sw.ctx.vadx_read_state(int(i)).astype(np.float64)
            e2, _ = scaled_err(fin[None], ref["final"][q][None])
            assert e2 <= TOL_STATE


@pytest.mark.parametrize("integrator,noise_off", [(1, False), (0, True)])
def test_euler_and_noise_free(oracle, integrator, noise_off):
    conn = inputs.synthetic_connectome(68)
    batch = inputs.grid_small().subset([1, 6])
    cfg = inputs.RunConfig(n_steps=500, n_trace_steps=500, seed=4)
    sw = run_gpu("literature-B", [conn], batch, cfg, trace=[0, 1], integrator=integrator,
                 noise_off=noise_off)
    ref = run_oracle(oracle, "literature-B", conn, batch, cfg, integrator=integrator,
                     noise_off=noise_off)
    for i in range(2):
        g = sw.ctx.vadx_read_trace(i, i, 500).astype(np.float64)
        e, where = scaled_err(g, ref["trace"][i])
        assert e <= TOL_STATE, f"{e:.3g} at {where}"


def test_chunked_launches_are_bit_identical():
    conn = inputs.synthetic_connectome(68)
    batch = inputs.grid_small()
    cfg = inputs.RunConfig(n_steps=1000, transient_steps=100)
    outs = []
    for chunk in (0, 96, 250):
        sw = run_gpu("literature-B", [conn], batch, cfg, chunk=chunk)
        outs.append((np.stack([sw.ctx.vadx_read_state(i) for i in range(8)]),
                     np.stack([sw.ctx.vadx_read_samples(i) for i in range(8)])))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


def test_degenerate_runs():
    conn = inputs.synthetic_connectome(68)
    batch = inputs.grid_small().subset([0])
    # no steps: FC of zero samples is the identity, flags report zero variance
    sw = run_gpu("literature-B", [conn], batch, inputs.RunConfig(n_steps=0))
    fc = sw.ctx.vadx_read_fc(0)
    assert np.array_equal(fc, np.eye(68, dtype=np.float32))
    assert sw.stats()[0]["flags"] & 4
    # transient covers the whole run: no samples
    sw = run_gpu("literature-B", [conn], batch, inputs.RunConfig(n_steps=200, transient_steps=200))
    assert sw.ctx.vadx_instance_shape(0)[1] == 0
    assert np.isfinite(sw.ctx.vadx_read_state(0)).all()


def test_invalid_arguments_rejected():
    sw = vadx.Sweep(0)
    conn = inputs.synthetic_connectome(20, seed=3)
    w = conn.weights.copy()
    w[0, 1] = -1.0
    with pytest.raises(vadx.VadxError) as ei:
        sw.ctx.vadx_add_connectome(w, conn.tract_mm)
    assert ei.value.status == vadx.VADX_E_ARG
    sw.add_connectome(conn)
    with pytest.raises(vadx.VadxError):
        sw.ctx.vadx_set_batch([0.1], [np.nan], [0.0], [4.0])
    with pytest.raises(vadx.VadxError):
        sw.ctx.vadx_set_batch([0.1], [0.0], [0.0], [-4.0])
    sw.ctx.vadx_set_batch([0.1], [0.0], [0.0], [4.0])
    run = vadx.make_run(inputs.RunConfig(n_steps=100))
    nbytes = sw.ctx.vadx_plan(run)
    import torch
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(vadx.VadxError) as ei:
        sw.ctx.vadx_integrate(run, ws.data_ptr(), nbytes // 2)
    assert ei.value.status == vadx.VADX_E_OOM
