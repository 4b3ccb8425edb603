"""The benchmark's rule for which Binder crossings it reports (CPU only).

A run supports an error estimate when Sokal's window for the integrated
autocorrelation time of M^2 converged, each jackknife block spans at least
10 tau kept sweeps and the discarded start at least 20 tau; a crossing of
two sizes is reported only when every run of both sizes passes.  Checked on
synthetic series: independent samples pass, a slowly drifting series fails,
and an unresolved pair yields a reason instead of a temperature."""
import math

import numpy as np
import pytest

import bench


@pytest.fixture(scope="module")
def I():
    from paper_1007_3726_amd import ising
    ising.lib()
    return ising


def _ar1_ints(phi, n, seed, scale=1000):
    rng = np.random.default_rng(seed)
    x = np.empty(n)
    x[0] = rng.standard_normal()
    s = math.sqrt(1 - phi * phi)
    for i in range(1, n):
        x[i] = phi * x[i - 1] + s * rng.standard_normal()
    return np.round(scale * (3.0 + x)).astype(np.int64)


def test_series_check(I):
    ok, tau, W = bench.series_check(I, _ar1_ints(0.0, 20000, 1), 2000, 20)
    assert ok and 0.3 < tau < 0.8 and W > 0
    # M^2 of 3 + AR(1): tau ~ (1 + phi) / (2 (1 - phi)) ~ 100 at phi = 0.99,
    # so blocks of 650 kept sweeps are < 10 tau
    ok, tau, W = bench.series_check(I, _ar1_ints(0.99, 15000, 2), 2000, 20)
    assert not ok and tau > 50
    # a long enough series with the same correlations passes
    ok, tau, W = bench.series_check(I, _ar1_ints(0.99, 400000, 3), 4000, 20)
    assert ok and 70 < tau < 140, tau
    # too short a discard for the correlations fails even with long blocks
    ok, tau, W = bench.series_check(I, _ar1_ints(0.99, 400000, 3), 500, 20)
    assert not ok


def test_crossings_only_where_resolved(I):
    T = np.linspace(2.2, 2.34, 8)
    Ua = 0.62 - 0.8 * (T - 2.27)       # smaller size: flatter
    Ub = 0.62 - 2.0 * (T - 2.27)       # larger size: steeper; they cross at 2.27
    B = 5
    rep_a = np.array([Ua + 0.001 * (b - 2) for b in range(B)])
    rep_b = np.array([Ub - 0.001 * (b - 2) for b in range(B)])
    curves = {8: (Ua[:, None], None, rep_a), 16: (Ub[:, None], None, rep_b)}
    good = {8: [(True, 1.0, 5)] * 3, 16: [(True, 2.0, 10)] * 3}
    out = bench.crossings_where_resolved(I, [8, 16], good, T, curves)
    assert out["8/16"]["resolved"] and abs(out["8/16"]["T"] - 2.27) < 1e-9
    bad = {8: [(True, 1.0, 5)] * 3, 16: [(True, 2.0, 10), (False, 900.0, -1), (True, 2.0, 10)]}
    out = bench.crossings_where_resolved(I, [8, 16], bad, T, curves)
    assert not out["8/16"]["resolved"] and "1 of 6 runs" in out["8/16"]["reason"]
    assert "L=16" in out["8/16"]["reason"] and "T" not in out["8/16"]
