"""Benchmark of the TVB-AdEx sweep hot path on one MI355X.

One step = one whole pass of the hot path over the uniform sweep: 4096
parameter combinations (64 x 64 inclusive grid of S in [0, 0.5] x b_e in
[0, 120], a_e = 0, v = 4 m/s) on one synthetic 68-region connectome, 100000
steps of 0.1 ms (10 s) of stochastic Heun each, then the Pearson FC over the
9000 post-transient 1 ms samples and the summary statistics. Inputs are
resident on the GPU before timing starts. Prints one JSON line.

The metric is instance-region-sim-s per wall-s: instances x regions x
simulated seconds / wall seconds.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MI355X_FP32_VECTOR_TFLOPS = 157.3   # published FP32 vector peak (packed FMA)
MI355X_HBM_GBPS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", choices=["uniform", "uneven", "small"], default="uniform")
    p.add_argument("--no-autotune", action="store_true",
                   help="keep the default launch shape instead of tuning it first")
    p.add_argument("--waves-per-simd", type=int, default=2, choices=[2, 3],
                   help="register budget of the integration kernel when not autotuning")
    p.add_argument("--wg-instances", type=int, default=0,
                   help="instances per workgroup when not autotuning (0 = as many as fit the lane budget)")
    p.add_argument("--lanes", type=int, default=0,
                   help="lane budget of every region-count class when not autotuning (0 = the "
                        "library's default, 256)")
    p.add_argument("--item-steps", type=int, default=0,
                   help="queue item length with --no-autotune (0 = 1000)")
    p.add_argument("--wave-slack", type=int, default=0, choices=[0, 1],
                   help="wave slack of the integration when not autotuning")
    p.add_argument("--tune-steps", type=int, default=24000,
                   help="steps of each autotuner trial run")
    p.add_argument("--tune-cache", default=os.path.join(tempfile.gettempdir(), "vadx_tune.json"))
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-instances", type=int, default=64)
    p.add_argument("--cpu-sample-steps", type=int, default=10000)
    p.add_argument("--traffic-json", default="",
                   help="HBM bytes per region-step measured with rocprofv3 counters (default: "
                        "profiles/traffic_<workload>.json, if present)")
    p.add_argument("--no-analysis", action="store_true",
                   help="skip the analysis-metric pass over the sweep's samples")
    p.add_argument("--analysis-reps", type=int, default=3)
    p.add_argument("--analysis-cpu-instances", type=int, default=8)
    p.add_argument("--no-guided", action="store_true",
                   help="skip the surrogate-guided sweep of the 32^4 grid (about a minute and a half)")
    p.add_argument("--no-uneven", action="store_true",
                   help="skip the uneven-batch object (8192 instances of 68/84/200 regions)")
    p.add_argument("--uneven-steps", type=int, default=3,
                   help="timed runs of the uneven batch (after one warm-up run)")
    p.add_argument("--plain-record", default=os.path.join(ROOT, "profiles", "plain_sweep_32x4.json"),
                   help="measured plain 32^4 sweep (wall time, full-grid errors), used while its "
                        "kernel source hash matches")
    p.add_argument("--write-plain-record", action="store_true",
                   help="also simulate the whole 32^4 grid plainly and write --plain-record")
    p.add_argument("--run-steps", type=int, default=0,
                   help="profiling only: shorten each run to this many steps (not a bench line)")
    p.add_argument("--copy-calibration-mib", type=int, default=0,
                   help="profiling only: first copy a buffer of this many MiB with torch (a "
                        "kernel of known traffic to scale FETCH_SIZE / WRITE_SIZE counters)")
    return p.parse_args()


def workload(name):
    from paper_2311_13337_amd import inputs
    conn = inputs.synthetic_connectome(68)
    if name == "uneven":
        conns = [conn, inputs.synthetic_connectome(84), inputs.synthetic_connectome(200)]
        return conns, inputs.grid_uneven(8192, seed=3), inputs.RUN_UNEVEN, (
            "uneven batch in one persistent launch: 8192 instances, a third each on 68-, 84- and "
            "200-region synthetic connectomes, S, b_e, a_e uniform in the sweep box, v uniform in "
            "1-10 m/s (ring depths 21-2001 steps); 50000 Heun steps of 0.1 ms (5 s), FC after a "
            "1 s transient")
    if name == "uniform":
        return [conn], inputs.grid_uniform(64, 64), inputs.RUN_UNIFORM, (
            "uniform sweep: 64x64 grid of (S in [0,0.5], b_e in [0,120] pA), a_e=0, v=4 m/s; "
            "4096 instances x 68 regions (synthetic connectome, 20% density, log-normal weights, "
            "10-200 mm tracts); 100000 Heun steps of 0.1 ms (10 s); FC over 9000 1-ms samples "
            "after a 1 s transient")
    return [conn], inputs.grid_small(), inputs.RUN_SMALL, (
        "small grid: 8 combos (S in {0.1,0.3} x b_e in {0,60} x a_e in {0,4}), v=4 m/s, "
        "68 regions, 10000 steps (1 s)")


def cpu_baseline(conns, batch, cfg, n_inst, n_steps):
    """The FP64 oracle on a bounded sample of the same workload (host cores)."""
    import numpy as np

    import oracle
    from paper_2311_13337_amd import inputs
    idx = np.linspace(0, len(batch) - 1, n_inst).round().astype(int)
    scfg = inputs.RunConfig(dt_ms=cfg.dt_ms, n_steps=n_steps, transient_steps=0,
                            tavg_steps=cfg.tavg_steps, seed=cfg.seed)
    threads = os.cpu_count() or 1
    units = 0.0
    t0 = time.perf_counter()
    for ci, conn in enumerate(conns):
        sel = idx[batch.conn[idx] == ci]
        if sel.size == 0:
            continue
        oracle.run(oracle.model(), scfg, conn, batch.subset(sel), inst_ids=sel, n_threads=threads)
        units += sel.size * conn.n * n_steps * cfg.dt_ms / 1000.0
    wall = time.perf_counter() - t0
    return {"value": units / wall, "unit": "instance-region-sim-s/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_inst} instances evenly spaced over the sweep x {n_steps} steps "
                      f"({n_steps * cfg.dt_ms / 1000:.1f} s simulated), FP64, one instance per "
                      f"thread, {wall:.1f} s wall"}


def measure(args, conns, batch, cfg, desc, workload_name, steps, warmup):
    """Plans (and autotunes) one workload, times `steps` whole runs after
    `warmup` untimed ones, and returns (line, sweep, context)."""
    import numpy as np
    import torch

    from paper_2311_13337_amd import vadx
    sw = vadx.Sweep(0)
    ids = [sw.add_connectome(c) for c in conns]
    sw.set_batch(batch, conn_ids=ids)
    run = vadx.make_run(cfg)
    sw.plan(run)
    sw.ctx.vadx_set_waves_per_simd(args.waves_per_simd)
    sw.ctx.vadx_set_launch(0, args.wg_instances, args.item_steps)
    sw.ctx.vadx_wave_slack(args.wave_slack)
    if args.lanes:
        for c in conns:
            sw.ctx.vadx_class_lanes(int(c.n), args.lanes)
    sw.plan(run)
    shape = {"instances_per_workgroup": args.wg_instances or "max",
             "lanes": args.lanes or "default",
             "item_steps": args.item_steps or 1000,
             "waves_per_simd": args.waves_per_simd, "autotuned": False}
    if not args.no_autotune:
        lanes, items, waves = sw.autotune(args.tune_cache, trial_steps=args.tune_steps)
        shape = {"lanes_per_workgroup": lanes, "item_steps": items, "waves_per_simd": waves,
                 "autotuned": True}
    ctx = sw.ctx
    shape.update(ctx.vadx_launch_info())
    shape["class_lanes"] = {int(c.n): ctx.vadx_class_lanes(int(c.n)) for c in conns}
    shape["wave_slack"] = ctx.vadx_wave_slack()
    for _ in range(warmup):
        sw.integrate()
    torch.cuda.synchronize()
    ctx.vadx_enable_timing(True)
    ctx.vadx_kernel_time()                      # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sw.integrate()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sw.sync()                                   # raises on a timed-out wait of the scheduler
    n_int, ms_int, n_fc, ms_fc = ctx.vadx_kernel_time()
    ctx.vadx_enable_timing(False)
    st = sw.stats()
    assert np.isfinite(st["fc_mean"]).all(), "non-finite FC mean"
    ms_per_step = (t1 - t0) * 1000.0 / steps
    # the same run replayed from a HIP graph (host clock; kernels not timed),
    # a few replays after the recording one
    g_steps = min(steps, 3)
    ctx.vadx_set_graph(True)
    sw.integrate()
    sw.sync()
    g0 = time.perf_counter()
    for _ in range(g_steps):
        sw.integrate()
    torch.cuda.synchronize()
    g1 = time.perf_counter()
    sw.sync()
    ctx.vadx_set_graph(False)
    graph_ms = (g1 - g0) * 1000.0 / g_steps
    n_inst = len(batch)
    regions = np.array([c.n for c in conns], np.float64)[batch.conn]
    region_total = float(regions.sum())
    sim_s = cfg.n_steps * cfg.dt_ms / 1000.0
    value = region_total * sim_s / (ms_per_step / 1000.0)

    # roofline of the integration kernel: the kernel's own arithmetic per
    # region-step (counted with an operation-counting scalar) plus 2 FLOPs per
    # delayed-coupling edge, times the region-steps of one launch
    f32, f64, trans = vadx.vadx_region_step_ops(vadx.VADX_HEUN)
    nnz = np.array([(c.weights != 0).sum() for c in conns], np.float64)
    edges = float(nnz[batch.conn].sum())
    flop_rs = f32 + f64 + 2.0 * edges / region_total + 1.0
    launches_per_step = n_int / steps
    rs_per_launch = region_total * cfg.n_steps / launches_per_step
    launch_ms = ms_int / n_int
    achieved = flop_rs * rs_per_launch / (launch_ms / 1000.0) / 1e12
    # HBM bytes of the integration kernel from rocprofv3 FETCH_SIZE/WRITE_SIZE
    # (copy-calibrated), stored per region-step for this kernel source and
    # launch shape (the block length and the workgroup's lanes change them)
    traffic = None
    traffic_json = args.traffic_json or os.path.join(ROOT, "profiles", f"traffic_{workload_name}.json")
    if os.path.exists(traffic_json):
        with open(traffic_json) as f:
            tj = json.load(f)
        here = {k: shape.get(k) for k in ("groups", "block_threads", "steps_per_block", "wave_slack")}
        same_shape = tj.get("shape") == here
        if tj.get("workload") == workload_name and tj.get("kernel_source_sha") == _src_sha() and same_shape:
            traffic = round(tj["bytes_per_region_step"] * rs_per_launch)
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": MI355X_FP32_VECTOR_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / MI355X_FP32_VECTOR_TFLOPS, 4),
            "traffic": traffic,
            "kernel": "integrate_persistent_kernel", "flop_per_region_step": round(flop_rs, 1),
            "transcendentals_per_region_step": trans,
            "launch_ms_avg": round(launch_ms, 3), "launches_per_step": launches_per_step,
            "fc_kernel_ms_per_step": round(ms_fc / max(n_fc, 1), 3)}
    flags = st["flags"].astype(np.uint32)
    out = {"metric": "instance-region-sim-s per wall-s", "value": round(value, 1),
           "unit": "instance-region-sim-s/s", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": desc, "instances": n_inst,
                      "regions": sorted({c.n for c in conns}),
                      "region_instances_total": int(region_total),
                      "steps_per_run": cfg.n_steps, "dt_ms": cfg.dt_ms,
                      "parallelism": "single GPU", "launch_shape": shape,
                      "timed_path": "eager persistent launch with HIP events around each kernel",
                      "graph_replay_ms_per_step": round(graph_ms, 3),
                      "clamp_flag_fraction": round(float(((flags & 2) != 0).mean()), 4),
                      "silent_fraction": round(float((st["rate_std_hz"] <= 1e-3).mean()), 4),
                      "nonfinite_fraction": round(float(((flags & 1) != 0).mean()), 4)},
           "roofline": roof}
    return out, sw, ctx


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the engine runs a sweep on a single MI355X "
              "(instances would shard across GPUs without communication). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2311_13337_amd import vadx

    conns, batch, cfg, desc = workload(args.workload)
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.run_steps > 0:
        import dataclasses
        cfg = dataclasses.replace(cfg, n_steps=args.run_steps,
                                  transient_steps=min(cfg.transient_steps, args.run_steps // 2))
        desc = f"[profiling run, {args.run_steps} steps] " + desc
    try:
        line = measure(args, conns, batch, cfg, desc, args.workload, args.steps, args.warmup)
    except vadx.VadxError as e:
        print(f"bench.py: the integration failed: {e}", file=sys.stderr)
        sys.exit(1)
    out, sw, ctx = line
    if not args.no_analysis and args.run_steps == 0:
        out["analysis"] = analysis_line(sw, conns, batch, cfg, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(conns, batch, cfg, args.cpu_sample_instances,
                                           args.cpu_sample_steps)
    if not args.no_uneven and args.workload == "uniform" and args.run_steps == 0:
        del sw, ctx
        torch.cuda.empty_cache()
        u_conns, u_batch, u_cfg, u_desc = workload("uneven")
        try:
            u, sw, ctx = measure(args, u_conns, u_batch, u_cfg, u_desc, "uneven", args.uneven_steps, 1)
        except vadx.VadxError as e:
            print(f"bench.py: the uneven-batch integration failed: {e}", file=sys.stderr)
            sys.exit(1)
        out["uneven"] = {k: u[k] for k in ("metric", "value", "unit", "steps", "warmup", "ms_per_step",
                                           "config", "roofline")}
    if not args.no_guided and args.workload == "uniform" and args.run_steps == 0:
        del sw, ctx
        torch.cuda.empty_cache()
        out["guided_vs_plain"] = guided_line(args.plain_record, args.write_plain_record)
    print(json.dumps(out), flush=True)


def analysis_line(sw, conns, batch, cfg, args):
    """The analysis metrics of Table 2 over the samples of the timed sweep
    (vadx_analyze on the integration workspace): time per pass over the whole
    batch, per-kernel times, the roofline of the dominant kernel, and the FP64
    oracle's time per instance on synthetic series of the same shape."""
    import numpy as np
    import torch

    from paper_2311_13337_amd import vadx
    ctx = sw.ctx
    n_inst = len(batch)
    n_max = max(c.n for c in conns)
    regions = np.array([c.n for c in conns], np.int64)[batch.conn]
    R = int(regions.sum())
    acfg = vadx.vadx_analysis_defaults()
    ns = cfg.n_samples
    Na = min(1 << (ns.bit_length() - 1), 16384)
    L = min(1024, Na)
    nb2 = L // 2 + 1
    n_seg = (Na - L) // (L // 2) + 1
    ws = torch.empty(vadx.vadx_analysis_ws_bytes(ns, n_max, R, acfg), dtype=torch.uint8,
                     device="cuda:0")
    out = vadx.analysis_out(n_inst)
    ctx.vadx_analyze(acfg, ws, out)              # warm-up
    torch.cuda.synchronize()
    ctx.vadx_enable_timing(True)
    vadx.analysis_kernel_time(ctx)               # reset
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = args.analysis_reps
    e0.record()
    for _ in range(reps):
        ctx.vadx_analyze(acfg, ws, out)
    e1.record()
    torch.cuda.synchronize()
    kt = vadx.analysis_kernel_time(ctx)
    ctx.vadx_enable_timing(False)
    ms = e0.elapsed_time(e1) / reps
    res = vadx.analysis_to_numpy(out)
    # algorithmic bytes (HBM) and FLOPs per pass, per kernel
    pairs = float(((regions * (regions - 1)) // 2).sum())
    work = {
        "an_transpose_kernel": {"bytes": 8.0 * Na * R},
        "an_welch_kernel": {"bytes": 4.0 * Na * R + 4.0 * nb2 * R,
                            "flop": R * n_seg * 5.0 * L * np.log2(L)},
        "an_hilbert_kernel": {"bytes": 12.0 * Na * R, "flop": R * 2 * 5.0 * Na * np.log2(Na)},
        "an_pli_kernel": {"bytes": 8.0 * Na * R, "flop": 3.0 * pairs * Na},
        "an_ud_kernel": {"bytes": 4.0 * Na * R},
        "an_final_kernel": {"bytes": 4.0 * nb2 * R},
    }
    kernels = {}
    for k, (nl, kms) in kt.items():
        d = {"ms": round(kms / reps, 3), "launches": nl // reps}
        if kms > 0:
            d["GB_s"] = round(work[k]["bytes"] / (kms / reps / 1000.0) / 1e9, 1)
            if "flop" in work[k]:
                d["TFLOP_s"] = round(work[k]["flop"] / (kms / reps / 1000.0) / 1e12, 2)
        kernels[k] = d
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    dms = kernels[dom]["ms"] / 1000.0
    if dom == "an_pli_kernel":
        # sign accumulation of Im(z_k conj z_l): plain VALU arithmetic
        ach = work[dom]["flop"] / dms / 1e12
        roof = {"bound": "alu", "achieved": round(ach, 3), "peak": MI355X_FP32_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / MI355X_FP32_VECTOR_TFLOPS, 4)}
    else:
        ach = work[dom]["bytes"] / dms / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": MI355X_HBM_GBPS, "unit": "GB/s",
                "frac": round(ach / MI355X_HBM_GBPS, 4)}
    roof["kernel"] = dom
    # BOLD of the same samples (Balloon-Windkessel, one thread per region)
    bcfg = vadx.vadx_bold_defaults()
    n_tr = int(ns * cfg.tavg_steps * cfg.dt_ms // bcfg.tr_ms)
    bout = torch.empty(max(R * n_tr, 1), dtype=torch.float32, device="cuda:0")
    ctx.vadx_bold(bcfg, bout)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        ctx.vadx_bold(bcfg, bout)
    e1.record()
    torch.cuda.synchronize()
    bold_ms = e0.elapsed_time(e1) / reps
    del bout
    # the oracle on synthetic series of the same shape (bounded sample)
    from oracle import analysis as oa

    from paper_2311_13337_amd import inputs
    S = inputs.synthetic_rate_series(args.analysis_cpu_instances, int(regions.min()), ns, seed=9)
    t0 = time.perf_counter()
    for i in range(S.shape[0]):
        oa.analyze_instance(S[i], cfg.tavg_steps * cfg.dt_ms)
    cpu_s = (time.perf_counter() - t0) / S.shape[0]
    return {"metric": "analysed instances per s", "value": round(n_inst / (ms / 1000.0), 1),
            "ms_per_pass": round(ms, 3), "instances": n_inst, "regions": R, "window": Na,
            "segment": L, "kernels": kernels, "roofline": roof,
            "bold": {"ms_per_pass": round(bold_ms, 3), "samples_per_region": ns,
                     "rk4_steps_per_s": round(R * ns / (bold_ms / 1000.0), 1),
                     "tr_ms": bcfg.tr_ms},
            "finite": bool(np.isfinite(res["psd_slope_a"]).all() and np.isfinite(res["mean_pli"]).all()),
            "mean_pli_mean": round(float(res["mean_pli"].mean()), 4),
            "cpu_oracle": {"s_per_instance": round(cpu_s, 4), "cores": 1, "kind": "oracle",
                           "sample": f"{S.shape[0]} synthetic instances of {int(regions.min())} "
                                     f"regions x {ns} samples (numpy FP64, one process)"}}


def guided_line(record_path, write_record=False):
    """The second half of the headline metric: the surrogate-guided sweep of the
    32^4 grid against the plain sweep, at the FC error bound. The plain sweep's
    wall time and the guided result's error over the whole grid come from a
    record of the measured full plain sweep while that record matches this
    kernel source and this guided result (same digest); otherwise the plain
    time is extrapolated from the plain runs of 4096 sampled grid points and
    the error is taken over those points. write_record: simulate the whole grid
    plainly as well and write the record (several minutes)."""
    import hashlib

    import numpy as np

    from paper_2311_13337_amd import guided
    try:
        res, data = guided.guided_sweep(guided.GuidedConfig(), plain_full=write_record,
                                        log=lambda m: print(m, file=sys.stderr, flush=True))
    except Exception as e:  # reported in the line; the throughput above stands
        return {"error": repr(e)}
    digest = hashlib.sha256(np.ascontiguousarray(data["guided"]).tobytes()).hexdigest()[:16]
    sec = res["seconds"]
    if write_record:
        fc = vadx_stat_index("fc_mean")
        e = np.abs(data["guided"][:, fc] - data["plain"][:, fc])
        active = data["plain"][:, vadx_stat_index("rate_std_hz")] > 1e-3
        rec = {"kernel_source_sha": _src_sha(), "guided_digest": digest,
               "workload": "32^4 grid over S [0,0.5] x b_e [0,120] x a_e [0,8] x v [1,10], 10-s runs "
                           "on the 68-region connectome, every grid point simulated plainly",
               "plain_s": round(sec["plain"], 3), "grid_points": res["grid_points"],
               "active_fraction": round(float(active.mean()), 4),
               "fc_mean_err_full_grid": {"p95": float(np.quantile(e, 0.95)), "max": float(e.max()),
                                         "mean": float(e.mean()),
                                         "p95_active": float(np.quantile(e[active], 0.95))
                                         if active.any() else 0.0},
               "guided_s": round(sec["guided_total"], 3), "refined_runs": res["refined"],
               "command": "python bench.py --no-uneven --no-analysis --no-cpu-baseline "
                          "--write-plain-record"}
        with open(record_path, "w") as f:
            json.dump(rec, f, indent=1)
    rec = None
    if os.path.exists(record_path):
        with open(record_path) as f:
            rec = json.load(f)
        if rec.get("kernel_source_sha") != _src_sha() or rec.get("guided_digest") != digest:
            rec = None
    plain_s = rec["plain_s"] if rec else sec["plain"]
    line = {"time_ratio_guided_over_plain": round(sec["guided_total"] / plain_s, 4),
            "guided_s": round(sec["guided_total"], 2), "plain_s": round(plain_s, 2),
            "plain_is_extrapolated": rec is None and sec["plain_is_extrapolated"],
            "fc_mean_err_p95": round(res["fc_mean_err"]["p95"], 4), "err_bound": 0.05,
            "passes_err_bound": res["passes_err_bound"],
            "refined_runs": res["refined"], "train_runs": res["train_sims"],
            "train_epochs": res["train"]["epochs"], "best_epoch": res["train"]["best_epoch"],
            "grid_points": res["grid_points"], "check_points": res["check_points"],
            "guided_digest": digest,
            "workload": "32^4 grid over S [0,0.5] x b_e [0,120] x a_e [0,8] x v [1,10], 10-s runs; "
                        "32768 training runs; top 5 % by the error network's prediction + 1 % audit, "
                        "then audit-driven refinement down that order"}
    if rec:
        line["full_grid"] = {k: rec[k] for k in ("fc_mean_err_full_grid", "active_fraction", "plain_s")}
        line["fc_mean_err_p95"] = round(rec["fc_mean_err_full_grid"]["p95"], 4)
        line["passes_err_bound"] = rec["fc_mean_err_full_grid"]["p95"] < 0.05
        line["check_points"] = rec["grid_points"]
    return line


def vadx_stat_index(name):
    from paper_2311_13337_amd import vadx
    return vadx.STAT_NAMES.index(name)


def _src_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "adex_model.h", "engine.h", "kmodel.h", "philox.h"):
        with open(os.path.join(ROOT, "paper_2311_13337_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
