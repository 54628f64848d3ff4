"""The integration kernel's wave synchronisation, checked by simulation on
the CPU (host logic of the kernel's design; no GPU).

Waves hold regions of instances; each instance's regions keep a ring of
excitatory-rate history, slot t mod D holding the rate after t steps. A wave
integrates blocks of B steps: at the block's start (step s) it reads, for every
edge of its regions, slots s + b - d (b < B, d the edge's delay); at the block's
end it writes slots s + 1 .. s + B of its own regions and publishes the number
of steps done. Before a block it waits until every wave sharing an instance
with it has published at least s + B - 1 - d_min steps (the newest slot its
reads reach). The simulation lets a random scheduler advance any wave whose
wait is satisfied and checks that every read returns the value written for
exactly the step it needs: written already, not yet overwritten.

Waves publish whole blocks, so a wave can run at most
L = B floor((d_min + 1) / B) <= d_min + 1 steps past the next block start of a
wave it waits for, which reads back d_max slots from there: a ring of
d_max + L + 1 slots is never overrun, in any schedule, and one slot fewer is
(the leading-wave schedules below find it). The kernel's rings have
d_max + d_min + 2 >= d_max + L + 1 slots, enough for every block length up to
d_min + 1 (its blocks with and without wave slack); a ring sized for waves one
block apart (d_max + B + 1) is overrun once blocks are shorter than d_min + 1.
"""
import numpy as np
import pytest


def simulate(waves, inst_regions, edges, B, D, n_steps, rng, greedy=None, wait_short=0):
    """waves: list of lists of regions; inst_regions: list of lists of
    regions (instances); edges: dict region -> list of (source, delay);
    wait_short: steps by which the waits fall short of the rule (0 = the
    kernel's rule); returns the number of reads that saw a wrong slot."""
    n_regions = sum(len(r) for r in inst_regions)
    inst_of = np.empty(n_regions, int)
    for i, regs in enumerate(inst_regions):
        inst_of[regs] = i
    dmin = min(d for es in edges.values() for _, d in es)
    # the waves each wave waits for: those sharing an instance with it
    insts = [set(inst_of[r] for r in w) for w in waves]
    nbrs = [[v for v in range(len(waves)) if v != w and insts[w] & insts[v]] for w in range(len(waves))]
    # the step whose rate a slot holds; every slot starts with the initial
    # rate, which is the rate of step 0 and of the history before it
    ring = np.zeros((n_regions, D), np.int64)
    published = [0] * len(waves)
    bad = 0
    while min(published) < n_steps:
        ready = []
        for w in range(len(waves)):
            s = published[w]
            if s >= n_steps:
                continue
            need = s + B - 1 - dmin - wait_short
            if all(published[v] >= need for v in nbrs[w]):
                ready.append(w)
        assert ready, "deadlock"
        if greedy == "max":          # let the wave furthest ahead run whenever it can
            w = max(ready, key=lambda v: (published[v], rng.random()))
        elif greedy == "chain":      # waves run in order, the first as far as it can
            w = min(ready)
        else:
            w = ready[rng.integers(len(ready))]
        s = published[w]
        nb = min(B, n_steps - s)
        # the gather: every read of the block, at its start
        for k in waves[w]:
            for j, d in edges[k]:
                for b in range(nb):
                    t = s + b - d
                    got = ring[j, t % D]
                    if got != max(t, 0):
                        bad += 1
        # the block's steps, then its writes and the publish
        for k in waves[w]:
            for t in range(s + 1, s + nb + 1):
                ring[k, t % D] = t
        published[w] = s + nb
    return bad


def network(rng, n_inst, n_per, dmin, dmax, deg=3):
    inst_regions = [list(range(i * n_per, (i + 1) * n_per)) for i in range(n_inst)]
    edges = {}
    for regs in inst_regions:
        for k in regs:
            src = rng.choice([j for j in regs if j != k], size=min(deg, len(regs) - 1), replace=False)
            ds = rng.integers(dmin, dmax + 1, size=len(src))
            ds[0] = dmin
            ds[-1] = dmax
            edges[k] = list(zip(src.tolist(), ds.tolist()))
    return inst_regions, edges


def chain_waves(inst_regions, per_wave):
    """Regions laid on consecutive lanes, per_wave regions to a wave (an
    instance may span waves, and a wave may hold parts of two instances)."""
    flat = [r for regs in inst_regions for r in regs]
    return [flat[i:i + per_wave] for i in range(0, len(flat), per_wave)]


CASES = [  # (instances, regions each, regions per wave, d_min, d_max, B)
    (3, 5, 4, 6, 20, 7),    # B = d_min + 1
    (3, 5, 4, 6, 20, 3),    # blocks of about half of d_min + 1 (wave slack)
    (2, 7, 3, 9, 31, 4),
    (2, 7, 3, 9, 31, 5),    # B divides d_min + 1 twice
    (4, 3, 2, 4, 12, 2),
    (1, 6, 2, 5, 9, 1),
]

SCHEDULES = ("max", "chain", None, "max", None)


def lead(dmin, B):
    return B * ((dmin + 1) // B)


def violations(case, D, seed, wait_short=0):
    n_inst, n_per, per_wave, dmin, dmax, B = case
    rng = np.random.default_rng(seed)
    inst_regions, edges = network(rng, n_inst, n_per, dmin, dmax, deg=4)
    waves = chain_waves(inst_regions, per_wave)
    return sum(simulate(waves, inst_regions, edges, B, D, 8 * D, rng, greedy=mode, wait_short=wait_short)
               for mode in SCHEDULES)


@pytest.mark.parametrize("case", CASES)
def test_kernel_rings_are_never_overrun(case):
    """Rings of d_max + d_min + 2 slots, as the planner sizes them."""
    _, _, _, dmin, dmax, B = case
    assert violations(case, dmax + dmin + 2, 5 + B) == 0


@pytest.mark.parametrize("case", CASES)
def test_exact_ring_bound(case):
    """d_max + L + 1 slots hold; one fewer is overrun."""
    _, _, _, dmin, dmax, B = case
    D = dmax + lead(dmin, B) + 1
    assert D <= dmax + dmin + 2
    assert violations(case, D, 17 + B) == 0
    assert violations(case, D - 1, 29 + B) > 0


def test_ring_sized_for_one_block_of_drift_is_overrun_by_short_blocks():
    """Rings of d_max + B + 1 slots hold only while waves stay a block apart;
    with blocks shorter than d_min + 1 the step-count waits let them drift
    further, which is why the rings are d_max + d_min + 2 deep."""
    case = (3, 5, 4, 6, 20, 3)
    assert violations(case, 20 + 3 + 1, 3) > 0


@pytest.mark.parametrize("case", CASES)
def test_earlier_waits_read_unwritten_slots(case):
    """Waits satisfied one publish earlier than the rule allows (the rule's
    target lowered just enough to reach the previous block end) let the
    leading wave read a slot before it is written, whatever the ring depth."""
    _, _, _, dmin, dmax, B = case
    short = B - (dmin + 1 - B) % B
    assert violations(case, dmax + dmin + 2 + 2 * B, 41 + B, wait_short=short) > 0
