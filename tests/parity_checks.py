"""Shared checks of the parity tests (no tests here): the re-anchored
comparison of a single-precision trajectory with the FP64 oracle's steps."""
import numpy as np

TOL_STATE = 1e-4
SLACK_REL = 2.0 ** -18      # input perturbation that measures a step's conditioning


def anchored_check(oracle, m, cfg, conn, batch, q, g, inst_id=None, integrator=0, noise_off=False):
    """Every step of trajectory g [steps, 8, n] (the state after each step)
    against one oracle step from g's previous state and rate history. Returns
    (err, slack_used): err[n] is the largest ratio, over states and regions,
    of |g - o| to TOL_STATE * max(|o|, rms of that state over the window)
    plus the step's own sensitivity: how far the oracle's step moves when its
    inputs (previous state and rate history) are perturbed by 2^-18 relative
    (random signs, three draws: 64 single-precision ulps, the input error
    that single-precision evaluation of erfc's far tail amounts to) -- at steps where the state sits near the moment
    bounds and one step cancels most of a rate, single-precision rounding of
    the inputs alone moves the result by more than 1e-4 of the state's scale.
    slack_used[n]: whether that sensitivity term exceeded the first."""
    o, _ = oracle.anchored_steps(m, cfg, conn, batch, q, g, inst_id=inst_id, integrator=integrator,
                                 noise_off=noise_off)
    rng = np.random.default_rng(12345)
    sens = np.zeros_like(o)
    for _ in range(3):
        gp = g * (1.0 + rng.choice([-1.0, 1.0], g.shape) * SLACK_REL)
        op, _ = oracle.anchored_steps(m, cfg, conn, batch, q, gp, inst_id=inst_id,
                                      integrator=integrator, noise_off=noise_off)
        sens = np.maximum(sens, np.abs(op - o))
    rms = np.sqrt((o ** 2).mean(axis=(0, 2), keepdims=True))
    base = TOL_STATE * np.maximum(np.abs(o), rms)
    den = base + sens
    den = np.where(den > 0, den, 1.0)
    err = (np.abs(g - o) / den).max(axis=(1, 2))
    return err, (sens > base).any(axis=(1, 2))
