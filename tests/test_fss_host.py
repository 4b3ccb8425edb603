"""The library's host-side FSS analysis (ising_fss_moments,
ising_binder_crossing) against the oracle on seeded inputs; argument checks.
Runs on the CPU (no device calls)."""
import math

import numpy as np
import pytest

from oracle import fss


@pytest.fixture(scope="module")
def I():
    from paper_1007_3726_amd import ising
    ising.lib()
    return ising


def test_moments_and_jackknife_match_the_oracle(I):
    rng = np.random.default_rng(11)
    nt, B = 9, 13
    sums = np.empty((nt, B, 5))
    sums[:, :, 0] = rng.uniform(50, 60, size=(nt, B))
    m = rng.uniform(100, 400, size=(nt, B))
    sums[:, :, 1] = sums[:, :, 0] * m
    sums[:, :, 2] = sums[:, :, 0] * m * m * rng.uniform(1.0, 1.2, size=(nt, B))
    sums[:, :, 3] = sums[:, :, 2] * m * m * rng.uniform(1.0, 1.4, size=(nt, B))
    sums[:, :, 4] = -sums[:, :, 0] * rng.uniform(1000, 2000, size=(nt, B))
    sites = rng.integers(64, 4096, size=nt)
    est, err, rep = I.fss_moments(sums, sites)
    for k in range(nt):
        e, r, u = fss.jackknife(sums[k], sites[k])
        assert np.allclose(est[k], e, rtol=1e-12, atol=0)
        assert np.allclose(err[k], r, rtol=1e-9, atol=1e-15)
        assert np.allclose(rep[k], u, rtol=1e-12, atol=0)


def test_crossing_matches_the_oracle(I):
    rng = np.random.default_rng(12)
    T = np.linspace(2.20, 2.34, 29)
    for trial in range(20):
        Tx = rng.uniform(2.21, 2.33)
        Ua = 0.61 - 1.5 * (T - Tx) + rng.normal(0, 0.004, size=len(T))
        Ub = 0.61 - 4.0 * (T - Tx) + rng.normal(0, 0.004, size=len(T))
        B = 8
        ra = Ua + rng.normal(0, 0.002, size=(B, len(T)))
        rb = Ub + rng.normal(0, 0.002, size=(B, len(T)))
        got = I.binder_crossing(T, Ua, Ub, ra, rb)
        want = fss.crossing_jackknife(T, Ua, Ub, ra, rb)
        for g, w in zip(got, want):
            assert (math.isnan(g) and math.isnan(w)) or g == pytest.approx(w, rel=1e-12, abs=1e-15)


def test_crossing_edges(I):
    T = np.linspace(0.0, 1.0, 11)
    assert all(math.isnan(v) for v in I.binder_crossing(T, T + 1.0, T))
    # straight lines: exact
    Ua = 0.6 - (T - 0.437)
    Ub = 0.6 - 2.0 * (T - 0.437)
    t, u, et, eu = I.binder_crossing(T, Ua, Ub)
    assert abs(t - 0.437) < 1e-14 and abs(u - 0.6) < 1e-14 and math.isnan(et)
    with pytest.raises(I.IsingError):
        I.binder_crossing(T[::-1], Ua, Ub)  # grid must ascend
    with pytest.raises(I.IsingError):
        I.binder_crossing(T[:1], Ua[:1], Ub[:1])  # need two points


def test_moments_argument_checks(I):
    with pytest.raises(I.IsingError):
        I.fss_moments(np.ones((2, 1, 5)), [16, 16])  # one block: no jackknife
    with pytest.raises(I.IsingError):
        I.fss_moments(np.ones((2, 3, 5)), [16, 0])


def _ar1(phi, n, seed):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0]
    s = math.sqrt(1.0 - phi * phi)
    for i in range(1, n):
        x[i] = phi * x[i - 1] + s * e[i]
    return x


@pytest.mark.parametrize("phi,n,c", [(0.0, 5000, 5.0), (0.7, 30000, 5.0), (0.95, 60000, 5.0),
                                     (0.95, 60000, 8.0), (0.999, 3000, 5.0)])
def test_autocorr_time_matches_the_oracle(I, phi, n, c):
    """The library forms C(t) by FFT, the oracle by direct sums: tau agrees to
    rounding (far below its statistical error) and the window exactly."""
    x = 1000.0 + 37.0 * _ar1(phi, n, int(phi * 1000) + n)
    got = I.autocorr_time(x, c)
    want = fss.autocorr_time(x, c)
    assert got[1] == want[1]
    assert abs(got[0] - want[0]) <= 1e-9 * max(1.0, abs(want[0]))


def test_autocorr_time_on_magnetisation_like_series(I):
    """Integer series of the kind the sweeps write (M^2 of a 64 x 64 lattice)."""
    rng = np.random.default_rng(5)
    M = np.cumsum(2 * rng.integers(-3, 4, size=20000)) % 4096 - 2048
    x = (M.astype(np.float64)) ** 2
    got = I.autocorr_time(x)
    want = fss.autocorr_time(x)
    assert got[1] == want[1] and abs(got[0] - want[0]) <= 1e-9 * max(1.0, abs(want[0]))
    assert I.autocorr_time(np.full(7, 2.0)) == (0.5, 0)
    assert I.autocorr_time(np.array([1.0, -1.0] * 8))[1] == 1


def test_autocorr_time_argument_checks(I):
    for bad in (([1.0], 5.0), ([1.0, 2.0], 0.0), ([1.0, 2.0], float("nan")),
                ([1.0, float("inf")], 5.0)):
        with pytest.raises(I.IsingError):
            I.autocorr_time(*bad)
