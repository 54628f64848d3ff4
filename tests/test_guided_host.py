"""Host logic of the guided sweep (no GPU): the audit-driven choice of how far
down the score ranking to refine."""
import numpy as np

from paper_2311_13337_amd.guided import refined_count


def test_refined_count_brute_force():
    """Against the definition evaluated by brute force: the smallest cut whose
    estimated unrefined-bad count is within the target."""
    rng = np.random.default_rng(1)
    for trial in range(200):
        n = int(rng.integers(100, 5000))
        k1 = int(rng.integers(0, n // 3))
        m = int(rng.integers(1, max(2, (n - k1) // 5)))
        score = rng.random(m)
        if trial % 3 == 0:
            score = np.round(score * 5) / 5                 # ties
        err = rng.random(m) * (1.5 * score)              # errors grow with the score
        bound, target = 0.5, float(rng.choice([0.0, 0.01, 0.05, 0.2]))
        got = refined_count(score, err, k1, n, bound, target)
        order = np.argsort(-score, kind="stable")
        per = (n - k1) / m
        want = None
        for j in range(m + 1):
            left_bad = int((err[order[j:]] > bound).sum())
            if left_bad * per <= target * n:
                want = min(n, k1 + int(np.ceil(j * per)))
                break
        assert got == want
        assert k1 <= got <= n


def test_refined_count_edges():
    s = np.array([0.9, 0.5, 0.1])
    assert refined_count(s, np.zeros(3), 10, 100, 0.05, 0.0) == 10        # nothing to fix
    assert refined_count(s, np.ones(3), 10, 100, 0.05, 0.0) == 100        # everything bad
    # only the top audit point is bad: cut right below it
    assert refined_count(s, np.array([1.0, 0, 0]), 10, 100, 0.05, 0.0) == 10 + 30
