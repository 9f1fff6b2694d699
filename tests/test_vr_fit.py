"""Variance-reduction fit (Sec. 2.4) on the host: no GPU needed.

The fit is parity-unpinned (the paper leaves the optimiser open); these tests
check its contract: exact recovery when the data come from the ansatz itself,
the identity for a flat histogram, the paper's parameter bounds, monotone
maps, and the fallback for an empty histogram.
"""

import numpy as np
import pytest

import oracle
import paper_1811_11720_amd as Q


def _inverse(a, x):
    lo, hi = np.zeros_like(x), np.ones_like(x)
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        val = np.array([oracle.vr_map(a, float(t))[0] for t in mid])
        m = val < x
        lo, hi = np.where(m, mid, lo), np.where(m, hi, mid)
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("a", [[1.2, -0.3, 0.15, 0.05, 0.6, 0.1], [2.5, -1.5, 0.1, 0.1, 0.7, 0.05]])
def test_fit_recovers_a_map_of_the_ansatz(a):
    bins = 512
    edges = np.arange(bins + 1) / bins
    cdf = _inverse(a, edges)  # CDF = p^-1 at the bin edges
    p, mask = Q.fit_vr_from_histogram(np.diff(cdf)[None, :])
    assert mask == 0
    ys = np.linspace(0, 1, 257)
    got = np.array([oracle.vr_map(p[0], y)[0] for y in ys])
    want = np.array([oracle.vr_map(a, y)[0] for y in ys])
    # the paper's stopping rule (step tolerance 3e-3, App. A.1) ends the fit
    # once steps are small, not at machine precision
    assert np.max(np.abs(got - want)) < 2e-4


def test_flat_histogram_gives_identity_and_bounds_hold():
    p, mask = Q.fit_vr_from_histogram(np.ones((3, 1024)))
    assert mask == 0
    ys = np.linspace(0, 1, 101)
    for j in range(3):
        assert p[j, 0] >= 1.001 and p[j, 1] <= -0.001
        got = np.array([oracle.vr_map(p[j], y)[0] for y in ys])
        assert np.max(np.abs(got - ys)) < 1e-6


def test_peaked_histogram_fit_is_monotone_with_endpoints():
    bins = 1024
    x = (np.arange(bins) + 0.5) / bins
    h = np.vstack([1.0 / (0.02 + x) ** 2, 1.0 / (1.02 - x) ** 1.5, np.exp(-8 * (x - 0.3) ** 2)])
    p, mask = Q.fit_vr_from_histogram(h)
    for j in range(3):
        if mask >> j & 1:
            continue
        assert oracle.vr_map(p[j], 0.0)[0] == 0.0
        assert abs(oracle.vr_map(p[j], 1.0)[0] - 1.0) < 1e-12
        d = [oracle.vr_map(p[j], y)[1] for y in np.linspace(0, 1, 513)]
        assert min(d) > 0


def test_empty_histogram_falls_back_to_identity():
    h = np.zeros((2, 64))
    h[1] = 1.0
    p, mask = Q.fit_vr_from_histogram(h)
    assert mask == 1
    assert list(p[0]) == [2.0, -1.0, 0.0, 0.0, 1.0, 0.0]
