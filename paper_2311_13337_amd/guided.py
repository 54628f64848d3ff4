"""Surrogate-guided sweep over (S, b_e, a_e, v) on one GPU.

The plain method simulates every point of a dense grid. The guided sweep
  1. simulates a training set of points drawn uniformly from the sweep box,
  2. trains the surrogate network on their statistics (vadx_mlp_train, early
     stopping on a held-out tenth), and a second network of the same shape on
     the surrogate's absolute errors over the training set,
  3. screens the whole grid with both: predicted statistics, and the
     predicted error of fc_mean as the refinement order (large where runs of
     one parameter point differ from run to run or the statistics change
     sharply; the surrogate's input-gradient norm of (sync_index, fc_mean) is
     the alternative order, cfg.score = "gradient"),
  4. simulates the points first in that order plus a random audit sample,
     each with the noise stream it has in the plain sweep (its grid index as
     noise key), so a refined point carries exactly its plain-sweep value,
  5. uses the audit sample -- simulated points drawn independently of the
     score -- to estimate, for each cut in that order, the fraction of the
     grid that would stay unrefined with an FC error above the bound, and
     refines further down the order until that estimate is below the target,
  6. keeps the predictions elsewhere.
The plain simulation stays the reference: the error of the guided result is
measured against plain runs of a random sample of grid points (bit-identical
to the full plain sweep at those points), and the plain sweep's time is the
measured per-instance time of the same simulations times the grid size.

All arithmetic runs in libvadx (simulation, training, screening, selection);
this module moves arrays between the calls and keeps the clock.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import inputs, vadx

STATS = vadx.STAT_NAMES
BOX = [inputs.SWEEP_BOX[a] for a in ("S", "b_e", "a_e", "v")]
TRAIN_KEY_BASE = 0x80000000          # noise keys of training runs (grid points use their index)
CHECK_SEED = 1


@dataclasses.dataclass
class GuidedConfig:
    grid_res: int = 32                 # points per axis of the grid
    n_train: int = 32768               # training simulations
    train_seed: int = 4
    top_frac: float = 0.05             # refined by predicted transition gradient
    audit_frac: float = 0.01           # random audit of the rest
    min_audit: int = 2000              # at least this many audit points (a 5 % exceed fraction
                                       # then has a binomial standard error below 0.5 points)
    audit_seed: int = 7
    run: inputs.RunConfig = inputs.RUN_UNIFORM
    batch: int = 1024
    lr: float = 1e-3
    max_epochs: int = 4000
    eval_every: int = 5
    patience: int = 400                # epochs without a better validation loss
    val_frac: float = 0.1
    split_seed: int = 0
    init_seed: int = 0
    n_check: int = 4096                # grid points simulated plainly to measure the error
    chunk: int = 16384                 # instances per simulation launch
    err_bound: float = 0.05
    target_exceed: float = 0.04        # audit estimate of the grid fraction above err_bound
    adaptive: bool = True
    score: str = "error"               # refinement order: "error" (a second network's predicted
                                       # error of fc_mean) or "gradient" (transition gradient)


class Simulator:
    """One context with the 68-region connectome; runs batches in chunks."""

    def __init__(self, conn, run_cfg, chunk, log=print):
        self.sw = vadx.Sweep(0)
        self.sw.add_connectome(conn)
        self.run = vadx.make_run(run_cfg)
        self.chunk = chunk
        self.log = log
        self.units_per_inst = conn.n * run_cfg.n_steps * run_cfg.dt_ms / 1000.0

    def __call__(self, batch, keys, label):
        n = len(batch)
        out = np.zeros((n, len(STATS)), np.float32)
        flags = np.zeros(n, np.uint32)
        t0 = time.perf_counter()
        for c0 in range(0, n, self.chunk):
            idx = np.arange(c0, min(n, c0 + self.chunk))
            self.sw.set_batch(batch.subset(idx), noise_keys=np.asarray(keys)[idx])
            self.sw.plan(self.run)
            self.sw.integrate()
            self.sw.sync()
            st = self.sw.stats()
            for j, name in enumerate(STATS):
                out[idx, j] = st[name]
            flags[idx] = st["flags"]
            self.log(f"[guided] {label}: {idx[-1] + 1}/{n} simulated "
                     f"({time.perf_counter() - t0:.1f} s)")
        return out, flags, time.perf_counter() - t0


def _points(batch):
    return np.stack([batch.S, batch.b_e, batch.a_e, batch.v], 1).astype(np.float32)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def train_surrogate(X, Y, cfg: GuidedConfig, log=print):
    """Trains the network on (X, Y) host arrays; returns (net, info)."""
    import torch
    n = X.shape[0]
    perm = np.random.default_rng(cfg.split_seed).permutation(n)
    n_val = max(1, int(round(cfg.val_frac * n)))
    va, tr = perm[:n_val], perm[n_val:]
    Xtr, Ytr, Xva, Yva = _dev(X[tr]), _dev(Y[tr]), _dev(X[va]), _dev(Y[va])
    lo = [b[0] for b in BOX]
    hi = [b[1] for b in BOX]
    net = vadx.Mlp(inputs.mlp_init_params(cfg.init_seed), lo, hi, lr=cfg.lr)
    net.fit_target_norm(Ytr)
    t0 = time.perf_counter()
    best, best_p, best_ep, ep = np.inf, net.params(), 0, 0
    history = []
    while ep < cfg.max_epochs:
        h = net.train(Xtr, Ytr, cfg.eval_every, cfg.batch)
        ep += cfg.eval_every
        val, _ = net.grad(Xva, Yva)
        history.append((ep, float(h[-1]), float(val)))
        if val < best:
            best, best_p, best_ep = val, net.params(), ep
        elif ep - best_ep >= cfg.patience:
            break
    net.set_params(best_p)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    log(f"[guided] trained {ep} epochs in {secs:.1f} s; best validation MSE {best:.4f} "
        f"(normalised units) at epoch {best_ep}")
    return net, {"epochs": ep, "best_epoch": best_ep, "val_mse": float(best), "seconds": secs,
                 "history": history}


def screen(net, grid_X):
    """Predicted statistics of every grid point and the screening score
    (device tensor)."""
    import torch
    t0 = time.perf_counter()
    Xd = _dev(grid_X)
    Y, _, score = net.predict(Xd, jacobian=False,
                              score_outputs=(STATS.index("sync_index"), STATS.index("fc_mean")))
    Yh = Y.cpu().numpy()
    torch.cuda.synchronize()
    return Yh, score, time.perf_counter() - t0


def train_error_net(net, X, Y, cfg: GuidedConfig, log=print):
    """A second network of the same shape, trained (same settings) on the
    surrogate's absolute errors over the training set: where the statistics
    vary from run to run (chaotic, noise-driven regimes) or change sharply, a
    prediction of the mean is far from any one run, and that is where
    refinement pays."""
    Yhat, _, _ = net.predict(_dev(X))
    R = np.abs(Yhat.cpu().numpy() - Y)
    err_net, info = train_surrogate(X, R, cfg, log=lambda m: log(m.replace("trained", "error net trained")))
    return err_net, info


def audit_fraction(cfg: GuidedConfig, n: int) -> float:
    """The audit's sampling fraction: cfg.audit_frac, raised on small grids so
    that the audit holds about cfg.min_audit points."""
    return float(min(1.0, max(cfg.audit_frac, cfg.min_audit / max(n, 1))))


def select(net, score, k, cfg: GuidedConfig):
    """Indices of the k largest scores plus the audit sample, and audit flags."""
    import torch
    n = score.numel()
    frac = audit_fraction(cfg, n)
    cap = k + int(n * frac * 1.5) + 1024
    sel = torch.empty(cap, dtype=torch.int64, device=score.device)
    aud = torch.empty(cap, dtype=torch.uint8, device=score.device)
    m = net.select(score, k, frac, cfg.audit_seed, sel, aud)
    return sel[:m].cpu().numpy(), aud[:m].cpu().numpy().astype(bool)


def refined_count(score_aud, err_aud, k1, n, bound, target):
    """Number k2 >= k1 of top-score points to simulate so that the grid points
    left unrefined with an error above `bound` are estimated to be at most a
    fraction `target` of the grid. The audit points are an independent random
    sample of the points outside the top k1 (each taken with the same
    probability), so the audit point ranked j by score stands for
    (n - k1) / len(audit) grid points, and the bad audit points ranked below it
    estimate the bad grid points a cut there would leave."""
    m = len(err_aud)
    order = np.argsort(-score_aud, kind="stable")
    bad = (err_aud[order] > bound).astype(np.int64)
    # bad_after[j] = bad audit points ranked j and below
    bad_after = np.concatenate([np.cumsum(bad[::-1])[::-1], [0]])
    per_audit = (n - k1) / m
    j = int(np.nonzero(bad_after * per_audit <= target * n)[0][0])
    return min(n, k1 + int(np.ceil(j * per_audit)))


def guided_sweep(cfg: GuidedConfig = GuidedConfig(), log=print, plain_full=False):
    """Runs the guided sweep and its check against the plain method. With
    plain_full the whole grid is also simulated plainly (small grids only)."""
    conn = inputs.synthetic_connectome(68)
    sim = Simulator(conn, cfg.run, cfg.chunk, log)
    grid = inputs.grid_4d(cfg.grid_res)
    G = _points(grid)
    n = len(grid)

    train = inputs.sample_box(cfg.n_train, seed=cfg.train_seed)
    Ytrain, ftrain, t_data = sim(train, TRAIN_KEY_BASE + np.arange(cfg.n_train), "training set")
    net, tinfo = train_surrogate(_points(train), Ytrain, cfg, log)
    Yhat, score, t_screen = screen(net, G)
    fc = STATS.index("fc_mean")
    if cfg.score == "error":
        err_net, einfo = train_error_net(net, _points(train), Ytrain, cfg, log)
        tinfo["seconds"] += einfo["seconds"]
        t0 = time.perf_counter()
        Rhat, _, _ = err_net.predict(_dev(G))
        score = Rhat[:, fc].contiguous()
        t_screen += time.perf_counter() - t0
    t0 = time.perf_counter()
    k1 = int(round(cfg.top_frac * n))
    idx, is_aud = select(net, score, k1, cfg)
    t_select = time.perf_counter() - t0
    log(f"[guided] screened {n} points in {t_screen:.2f} s; refining {len(idx)} "
        f"({int((~is_aud).sum())} by score, {int(is_aud.sum())} audit)")
    Yref, fref, t_refine = sim(grid.subset(idx), idx, "refinement")
    k2 = k1
    if cfg.adaptive and is_aud.any():
        t0 = time.perf_counter()
        aud = idx[is_aud]
        err_aud = np.abs(Yhat[aud, fc] - Yref[is_aud, fc])
        k2 = refined_count(score[aud].cpu().numpy(), err_aud, k1, n, cfg.err_bound,
                           cfg.target_exceed)
        if k2 > k1:
            idx2, is_aud2 = select(net, score, k2, cfg)
            new = np.setdiff1d(idx2, idx, assume_unique=True)
            t_select += time.perf_counter() - t0
            log(f"[guided] audit: {int((err_aud > cfg.err_bound).sum())}/{len(aud)} audit points "
                f"above {cfg.err_bound}; refining the top {k2 / n:.1%} ({len(new)} more runs)")
            Ynew, fnew, t_more = sim(grid.subset(new), new, "refinement, second pass")
            t_refine += t_more
            idx = np.concatenate([idx, new])
            Yref = np.concatenate([Yref, Ynew])
            fref = np.concatenate([fref, fnew])
            is_aud = np.concatenate([is_aud, np.zeros(len(new), bool)])
        else:
            t_select += time.perf_counter() - t0
    guided = Yhat.copy()
    guided[idx] = Yref
    refined = np.zeros(n, bool)
    refined[idx] = True
    t_guided = t_data + tinfo["seconds"] + t_screen + t_select + t_refine

    if plain_full:
        chk = np.arange(n)
    else:
        chk = np.sort(np.random.default_rng(CHECK_SEED).choice(n, min(cfg.n_check, n),
                                                              replace=False))
    Yplain, _, t_check = sim(grid.subset(chk), chk, "plain check")
    sec_per_inst = (t_refine + t_check) / (len(idx) + len(chk))
    t_plain = t_check if plain_full else sec_per_inst * n

    def errs(col):
        e = np.abs(guided[chk, col] - Yplain[:, col])
        e_pred = np.abs(Yhat[chk, col] - Yplain[:, col])
        return {"p95": float(np.quantile(e, 0.95)), "max": float(e.max()),
                "mean": float(e.mean()), "surrogate_only_p95": float(np.quantile(e_pred, 0.95))}

    res = {
        "grid_points": n, "train_sims": cfg.n_train, "refined": int(len(idx)),
        "refined_audit": int(is_aud.sum()), "check_points": int(len(chk)),
        "check_points_refined": int(refined[chk].sum()),
        "fc_mean_err": errs(STATS.index("fc_mean")),
        "fc_sc_corr_err": errs(STATS.index("fc_sc_corr")),
        "sync_index_err": errs(STATS.index("sync_index")),
        "top_fraction_refined": k2 / n,
        "seconds": {"train_data": t_data, "train": tinfo["seconds"], "screen": t_screen,
                    "select": t_select, "refine": t_refine, "guided_total": t_guided,
                    "plain": t_plain, "plain_is_extrapolated": not plain_full,
                    "plain_sec_per_instance": sec_per_inst},
        "time_ratio_guided_over_plain": t_guided / t_plain,
        "train": {k: v for k, v in tinfo.items() if k != "history"},
        "flags_nonfinite": int(((ftrain & 1) != 0).sum() + ((fref & 1) != 0).sum()),
    }
    res["passes_err_bound"] = res["fc_mean_err"]["p95"] < cfg.err_bound
    return res, {"guided": guided, "pred": Yhat, "idx": idx, "check": chk, "plain": Yplain,
                 "grid": G, "train_X": _points(train), "train_Y": Ytrain,
                 "score": score.cpu().numpy()}
