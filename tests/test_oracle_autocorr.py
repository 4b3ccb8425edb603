"""Pins the oracle's integrated autocorrelation time (CPU only).

For a stationary AR(1) series x_{i+1} = phi x_i + sqrt(1 - phi^2) e_i the
autocorrelation is exactly rho(t) = phi^t, so the integrated time is
tau = 1/2 + phi / (1 - phi) = (1 + phi) / (2 (1 - phi)).  Sokal's windowed
estimate has a statistical error of about tau sqrt(2 (2W + 1) / n) and a
truncation bias of phi^(W+1) / (1 - phi), both small here.  Exact cases: an
alternating series has rho(t) = (-1)^t up to its (n - t) normalisation, a
constant series has no fluctuation.  Forgetting the 1/2, normalising C(t) by
n instead of n - t on a short series, or summing rho from t = 0 fails these.
"""
import math

import numpy as np
import pytest

from oracle import fss


def _ar1(phi, n, seed):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0]
    s = math.sqrt(1.0 - phi * phi)
    for i in range(1, n):
        x[i] = phi * x[i - 1] + s * e[i]
    return x


@pytest.mark.parametrize("phi,seed", [(0.0, 1), (0.5, 2), (0.9, 3), (0.98, 4)])
def test_ar1_series_of_known_tau(phi, seed):
    n = 1_000_000
    x = _ar1(phi, n, seed)
    tau, W = fss.autocorr_time(x)
    exact = (1 + phi) / (2 * (1 - phi))
    assert W > 0 and W >= 5 * tau
    sigma = exact * math.sqrt(2 * (2 * W + 1) / n)
    bias = phi ** (W + 1) / (1 - phi)
    assert abs(tau - exact) <= 5 * sigma + bias, (tau, exact, sigma)


def test_mean_error_from_tau_matches_block_spread():
    """sqrt(2 tau C(0) / n) is the error of the mean: compare with the
    spread of the means of 400 independent AR(1) series."""
    phi, n = 0.8, 20_000
    means, taus = [], []
    for s in range(400):
        x = _ar1(phi, n, 100 + s)
        means.append(x.mean())
        if s < 20:
            taus.append(fss.autocorr_time(x)[0])
    tau = float(np.mean(taus))
    predicted = math.sqrt(2 * tau / n)  # C(0) = 1 for this normalisation
    observed = float(np.std(means, ddof=1))
    assert 0.85 < observed / predicted < 1.15, (observed, predicted)


def test_exact_small_cases():
    # alternating: C(t) = (-1)^t, so tau(1) = 1/2 - 1 < 0 and W = 1
    tau, W = fss.autocorr_time(np.array([1.0, -1.0] * 8))
    assert W == 1 and tau == pytest.approx(-0.5, abs=1e-15)
    # constant: no fluctuation
    assert fss.autocorr_time(np.full(10, 3.0)) == (0.5, 0)
    # four samples, hand computed: y = (-1.5, -0.5, 0.5, 1.5), C(0) = 5/4,
    # C(1) = (0.75 - 0.25 + 0.75) / 3 = 5/12, rho(1) = 1/3: tau(1) = 5/6,
    # 1 < 5 tau(1); C(2) = (-0.75 - 0.75) / 2 = -3/4, rho(2) = -3/5:
    # tau(2) = 7/30 and 2 >= 5 * 7/30
    tau, W = fss.autocorr_time(np.array([1.0, 2.0, 3.0, 4.0]))
    assert W == 2 and tau == pytest.approx(7 / 30, abs=1e-15)


def test_too_short_for_its_correlations():
    x = _ar1(0.999, 2000, 9)
    tau, W = fss.autocorr_time(x)
    assert W == -1 and tau > 20
    with pytest.raises(ValueError):
        fss.autocorr_time([1.0])
