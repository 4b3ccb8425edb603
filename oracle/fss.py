"""Finite-size-scaling analysis of per-sweep (E, M) series, written plainly.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
it; the product path never imports it.

The paper locates T_C from the Binder cumulant U4 = 1 - <M^4> / (3 <M^2>^2)
(section 2, Eq. (2)): U4 curves of different linear sizes cross at T_C.
Three textbook tools turn the simulated series into that crossing:

* single-histogram reweighting (A. M. Ferrenberg and R. H. Swendsen, Phys.
  Rev. Lett. 61, 2635 (1988)): a series sampled at beta0 gives averages at a
  nearby beta with weights w_t = exp(-(beta - beta0) E_t);
* the delete-one-block jackknife (B. Efron, 1982) for the statistical error
  of non-linear estimators such as U4;
* the crossing of two U4 curves on a common temperature grid, by linear
  interpolation between the grid points that bracket the first sign change.

Definitions shared with the library (they define the results, so both sides
follow them; the code is written separately):

* kept samples are t = discard .. n-1; sample j = t - discard belongs to
  block floor(j * B / count), count = n - discard;
* x_t = -(beta - beta0) * (E_t - E_ref) with E_ref = E of the first kept
  sample, w_t = exp(x_t - max_t x_t);
* per block the five sums  S0 = sum w,  S1 = sum w |M|,  S2 = sum w M^2,
  S3 = sum w M^4,  S4 = sum w E, with m = double(M), m2 = m * m,
  m4 = m2 * m2 and e = double(E);
* from sums S: <M^2> = S2 / S0, <M^4> = S3 / S0, U4 = 1 - <M^4> / (3 <M^2>^2),
  e = S4 / (S0 N), |m| = S1 / (S0 N);
* jackknife: replica b uses the totals minus block b; error =
  sqrt((B - 1) / B * sum_b (q_b - mean_b q_b)^2);
* crossing: d_k = Ua_k - Ub_k with Ua the smaller and Ub the larger size on
  an ascending grid T_k; the first k with d_k < 0 <= d_{k+1} gives
  T* = T_k + (T_{k+1} - T_k) d_k / (d_k - d_{k+1}) and U* = Ua interpolated
  at T*; no such k gives NaN.  (Below T_C the larger lattice has the larger
  U4, above it the smaller.)
"""
import math

import numpy as np


def reweight_sums(E, M, discard, beta0, beta, nblocks):
    """Per-block reweighted sums [nblocks][5] and the shift max_t x_t."""
    E = np.asarray(E, dtype=np.int64)[discard:]
    M = np.asarray(M, dtype=np.int64)[discard:]
    count = len(E)
    if count < nblocks or nblocks < 1:
        raise ValueError("need at least one kept sample per block")
    x = -(beta - beta0) * (E - E[0]).astype(np.float64)
    shift = float(x.max())
    w = np.exp(x - shift)
    m = M.astype(np.float64)
    m2 = m * m
    m4 = m2 * m2
    e = E.astype(np.float64)
    block = (np.arange(count, dtype=np.int64) * nblocks) // count
    out = np.zeros((nblocks, 5))
    for b in range(nblocks):
        sel = block == b
        ws = w[sel]
        out[b] = [ws.sum(), (ws * np.abs(m[sel])).sum(), (ws * m2[sel]).sum(),
                  (ws * m4[sel]).sum(), (ws * e[sel]).sum()]
    return out, shift


def quantities(S, N):
    """(U4, <E>/N, <|M|>/N) from one set of the five sums."""
    S0, S1, S2, S3, S4 = S
    m2 = S2 / S0
    m4 = S3 / S0
    return np.array([1.0 - m4 / (3.0 * m2 * m2), S4 / (S0 * N), S1 / (S0 * N)])


def jackknife(sums, N):
    """Estimates from the totals, their jackknife errors and the U4 replicas."""
    sums = np.asarray(sums, dtype=np.float64)
    B = sums.shape[0]
    total = sums.sum(axis=0)
    est = quantities(total, N)
    reps = np.array([quantities(total - sums[b], N) for b in range(B)])
    mean = reps.mean(axis=0)
    err = np.sqrt((B - 1) / B * ((reps - mean) ** 2).sum(axis=0))
    return est, err, reps[:, 0]


def crossing(T, Ua, Ub):
    """First crossing of Ua (smaller size) and Ub (larger size): (T*, U*)."""
    T = np.asarray(T, dtype=np.float64)
    d = np.asarray(Ua, dtype=np.float64) - np.asarray(Ub, dtype=np.float64)
    for k in range(len(T) - 1):
        if d[k] < 0.0 <= d[k + 1]:
            f = d[k] / (d[k] - d[k + 1])
            Tx = T[k] + (T[k + 1] - T[k]) * f
            Ux = Ua[k] + (Ua[k + 1] - Ua[k]) * f
            return float(Tx), float(Ux)
    return math.nan, math.nan


def crossing_jackknife(T, Ua, Ub, Ua_rep, Ub_rep):
    """Crossing from the full curves and its jackknife error from the B
    replica curves (rows of Ua_rep / Ub_rep): (T*, U*, err T*, err U*)."""
    Tx, Ux = crossing(T, Ua, Ub)
    B = len(Ua_rep)
    reps = np.array([crossing(T, Ua_rep[b], Ub_rep[b]) for b in range(B)])
    if np.isnan(reps).any():
        return Tx, Ux, math.nan, math.nan
    mean = reps.mean(axis=0)
    err = np.sqrt((B - 1) / B * ((reps - mean) ** 2).sum(axis=0))
    return Tx, Ux, float(err[0]), float(err[1])


def autocorr_time(x, c=5.0):
    """Integrated autocorrelation time of a series, with the automatic
    window of A. D. Sokal (Monte Carlo methods in statistical mechanics,
    Cargese lectures 1996, section 3): with the sample mean removed,
      C(t) = sum_{i < n - t} y_i y_{i+t} / (n - t),  rho(t) = C(t) / C(0),
      tau(W) = 1/2 + sum_{t=1}^{W} rho(t),
    and W the smallest window in 1 .. floor(n / 2) with W >= c tau(W).
    Returns (tau(W), W); (tau(floor(n / 2)), -1) when no window qualifies
    (the series is too short for its correlations); (0.5, 0) for a constant
    series.  The error of a mean of n samples is then sqrt(2 tau C(0) / n)."""
    y = np.asarray(x, dtype=np.float64)
    n = len(y)
    if n < 2:
        raise ValueError("need at least two samples")
    y = y - y.mean()
    c0 = float(np.dot(y, y)) / n
    if c0 == 0.0:
        return 0.5, 0
    tau = 0.5
    for W in range(1, n // 2 + 1):
        tau += float(np.dot(y[:n - W], y[W:])) / (n - W) / c0
        if W >= c * tau:
            return tau, W
    return tau, -1
