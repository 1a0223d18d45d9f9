"""Host-side pieces of the benchmark (CPU only): the exact one-sided
Wilcoxon signed-rank test of the processing-time hypothesis sweep."""
import numpy as np

import bench


def test_signed_rank_closed_forms():
    n = 14
    a, b = np.arange(1, n + 1, dtype=float), np.zeros(n)
    assert bench.signed_rank_p_greater(a, b) == 2.0 ** -n          # every sign positive: one pattern of 2^n
    assert bench.signed_rank_p_greater(b, a) == 1.0                # every sign negative
    assert bench.signed_rank_p_greater(a, a) == 1.0                # no nonzero difference
    # one negative difference of rank 1: W+ = n(n+1)/2 - 1, reached by 2 patterns
    d = np.arange(1, n + 1, dtype=float)
    d[0] = -1
    assert bench.signed_rank_p_greater(d, np.zeros(n)) == 2 * 2.0 ** -n


def test_signed_rank_ties_and_symmetry():
    # tied magnitudes share their average rank; a symmetric sample sits at p > 1/2
    d = np.array([1.0, -1.0, 2.0, -2.0, 3.0, -3.0])
    p = bench.signed_rank_p_greater(d, np.zeros(6))
    assert 0.5 < p < 0.7
    g = np.random.default_rng(3)
    for _ in range(5):
        x = g.integers(-5, 6, 10).astype(float)
        p1 = bench.signed_rank_p_greater(x, np.zeros(10))
        p2 = bench.signed_rank_p_greater(-x, np.zeros(10))
        k = (x != 0).sum()
        # P(W+ >= w) + P(W+ <= w) = 1 + P(W+ = w) >= 1 under the symmetric null
        assert p1 + p2 >= 1.0 - 1e-12 or k == 0
