"""Pins of the oracle's finite-size-scaling analysis (oracle/fss.py).

* reweighting the complete 4 x 4 state list from beta0 = 0 (where every
  state is equally likely) must give the exact canonical averages at any
  temperature, computed here by brute force over the same 2^16 states;
* reweighting to beta0 itself is the plain sample mean; a constant energy
  offset changes nothing; the blocks partition the kept samples;
* a long i.i.d. sample of the exact 4 x 4 distribution at one temperature,
  reweighted to another, agrees with the exact values there within errors;
* the jackknife error of a linear statistic over equal blocks equals the
  closed-form standard error of the block means; for U4 it matches the
  spread of independent replicas;
* crossings of straight lines are exact; no sign change gives NaN; the
  first change from Ua < Ub to Ua >= Ub is the one reported;
* the whole chain on oracle Metropolis runs of L = 8 and 16 puts the
  Binder crossing near T_C = 2/ln(1 + sqrt 2).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import fss
import physics
import workloads


@pytest.fixture(scope="module")
def states4():
    return physics.enumerate_states(4)


def exact_canonical(E, M, T, N):
    """Brute-force canonical averages over an explicit state list."""
    w = np.exp(-(E - E.min()) / T)
    Z = w.sum()
    m = M.astype(np.float64)
    return {"e": (w * E).sum() / Z / N, "am": (w * np.abs(m)).sum() / Z / N,
            "m2": (w * m * m).sum() / Z, "m4": (w * m ** 4).sum() / Z}


@pytest.mark.parametrize("T", [2.0, 2.269185, 3.0, 5.0])
def test_reweighting_the_complete_state_list_is_exact(states4, T):
    E, M = states4
    N = 16
    sums, shift = fss.reweight_sums(E, M, 0, 0.0, 1.0 / T, 16)
    tot = sums.sum(axis=0)
    ex = exact_canonical(E, M, T, N)
    u4_exact = 1.0 - ex["m4"] / (3.0 * ex["m2"] ** 2)
    u4, e, am = fss.quantities(tot, N)
    assert abs(u4 - u4_exact) < 1e-12
    assert abs(e - ex["e"]) < 1e-12
    assert abs(am - ex["am"]) < 1e-12
    assert abs(tot[2] / tot[0] - ex["m2"]) < 1e-10 * ex["m2"]
    # and against the independent enumeration helper of the oracle pins
    ref = physics.exact_moments(4, T)
    assert abs(u4 - ref["u4"]) < 1e-12 and abs(e - ref["e"]) < 1e-12
    assert shift == pytest.approx(-(1.0 / T) * float(E.min() - E[0]))


def test_reweighting_to_the_same_beta_is_the_sample_mean():
    rng = np.random.default_rng(1)
    E = -4 * rng.integers(0, 500, size=1003)
    M = 2 * rng.integers(-300, 300, size=1003)
    B, d = 7, 3
    sums, shift = fss.reweight_sums(E, M, d, 0.44, 0.44, B)
    assert shift == 0.0
    cnt = len(E) - d
    sizes = sums[:, 0]
    assert sizes.sum() == cnt and set(sizes) <= {cnt // B, cnt // B + 1}
    m = M[d:].astype(np.float64)
    assert sums[:, 2].sum() == pytest.approx((m * m).sum(), rel=1e-14)
    assert sums[:, 4].sum() == pytest.approx(E[d:].astype(np.float64).sum(), rel=1e-14)
    # blocks are consecutive: block b ends where block b+1 begins
    starts = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    for b in range(B):
        seg = m[starts[b]:starts[b + 1]]
        assert sums[b, 1] == pytest.approx(np.abs(seg).sum(), rel=1e-14)


def test_energy_offset_changes_no_ratio():
    rng = np.random.default_rng(2)
    E = -4 * rng.integers(100, 400, size=600)
    M = 2 * rng.integers(-200, 200, size=600)
    a, _ = fss.reweight_sums(E, M, 0, 0.40, 0.43, 5)
    b, _ = fss.reweight_sums(E - 400, M, 0, 0.40, 0.43, 5)
    ra = a[:, 1:4] / a[:, :1]
    rb = b[:, 1:4] / b[:, :1]
    assert np.allclose(ra, rb, rtol=1e-12)
    assert np.allclose(a[:, 4] / a[:, 0] - 400, b[:, 4] / b[:, 0], rtol=1e-12)


def test_reweighted_iid_sample_agrees_with_exact_values(states4):
    E, M = states4
    T0, T1 = 2.3, 2.2
    w = np.exp(-(E - E.min()) / T0)
    p = w / w.sum()
    rng = np.random.default_rng(20100707)
    idx = rng.choice(len(E), size=400_000, p=p)
    sums, _ = fss.reweight_sums(E[idx], M[idx], 0, 1.0 / T0, 1.0 / T1, 40)
    est, err, _ = fss.jackknife(sums, 16)
    ex = exact_canonical(E, M, T1, 16)
    u4_exact = 1.0 - ex["m4"] / (3.0 * ex["m2"] ** 2)
    for got, e, want in zip(est, err, [u4_exact, ex["e"], ex["am"]]):
        assert 0 < e < 0.01
        assert abs(got - want) < 5 * e


def test_jackknife_of_a_linear_statistic_is_the_block_standard_error():
    rng = np.random.default_rng(3)
    B = 10
    M = 2 * rng.integers(1, 1000, size=B * 97)  # positive, so |M| = M
    E = np.full_like(M, -40)
    sums, _ = fss.reweight_sums(E, M, 0, 0.5, 0.5, B)
    N = 100
    est, err, _ = fss.jackknife(sums, N)
    bm = M.reshape(B, -1).mean(axis=1) / N
    se = math.sqrt(((bm - bm.mean()) ** 2).sum() / (B * (B - 1)))
    assert est[2] == pytest.approx(M.mean() / N, rel=1e-13)
    assert err[2] == pytest.approx(se, rel=1e-10)
    assert err[1] < 1e-12  # constant energy: only rounding


def test_jackknife_error_of_u4_matches_replica_spread():
    rng = np.random.default_rng(4)
    B, n, reps = 20, 4000, 300
    u, e = [], []
    for _ in range(reps):
        M = np.round(rng.normal(0.0, 300.0, size=n)).astype(np.int64)
        sums, _ = fss.reweight_sums(np.zeros(n, dtype=np.int64), M, 0, 0.3, 0.3, B)
        est, err, _ = fss.jackknife(sums, 1024)
        u.append(est[0])
        e.append(err[0])
    spread = np.std(u, ddof=1)
    assert 0.8 < np.mean(e) / spread < 1.25
    assert abs(np.mean(u)) < 4 * spread / math.sqrt(reps)  # Gaussian: U4 = 0


def test_crossing_of_straight_lines_is_exact():
    T = np.linspace(2.20, 2.34, 15)
    Tx = 2.2713
    Ua = 0.6 - 1.0 * (T - Tx)
    Ub = 0.6 - 3.0 * (T - Tx)
    t, u = fss.crossing(T, Ua, Ub)
    assert abs(t - Tx) < 1e-13 and abs(u - 0.6) < 1e-13


def test_no_crossing_gives_nan_and_the_first_upward_change_is_taken():
    T = np.linspace(0.0, 1.0, 11)
    assert all(math.isnan(v) for v in fss.crossing(T, T + 1.0, T))
    d = np.array([-1, 1, -1, -1, 1, 1, 1, 1, 1, 1, 1], dtype=float)
    t, _ = fss.crossing(T, d, np.zeros(11))
    assert t == pytest.approx(0.05)
    # a change from >= to < (the wrong direction) is not a crossing
    assert math.isnan(fss.crossing(T, -T + 0.55, np.zeros(11))[0])


def test_crossing_jackknife_error_closed_form():
    T = np.linspace(2.2, 2.34, 8)
    B = 6
    shifts = np.array([0.001, -0.002, 0.0005, 0.0, 0.003, -0.001])
    base = 2.27
    Ua = 0.6 - (T - base)
    Ub = 0.6 - 2 * (T - base)
    Ua_rep = [0.6 - (T - base - s) for s in shifts]
    Ub_rep = [0.6 - 2 * (T - base - s) for s in shifts]
    t, u, et, eu = fss.crossing_jackknife(T, Ua, Ub, Ua_rep, Ub_rep)
    want = math.sqrt((B - 1) / B * ((shifts - shifts.mean()) ** 2).sum())
    assert t == pytest.approx(base, abs=1e-13)
    assert et == pytest.approx(want, rel=1e-9)
    assert eu < 1e-12


def test_binder_crossing_of_oracle_runs_is_near_tc():
    """L = 8 and 16, six temperatures around T_C, 60000 sweeps each: the
    crossing of the reweighted U4 curves lies within 0.03 (plus 4 errors)
    of T_C."""
    temps = np.linspace(2.15, 2.40, 6)
    fine = np.linspace(2.15, 2.40, 51)
    n, d, B = 60_000, 6_000, 20
    saved = oracle.get_threads()
    oracle.set_threads(1)
    try:
        curves = {}
        for L in (8, 16):
            est = np.empty(len(fine))
            rep = np.empty((B, len(fine)))
            series = []
            for i, T in enumerate(temps):
                _, EM = oracle.run(L, 1.0 / T, 100 + i, L, workloads.INIT_HOT, n)
                series.append(EM)
            for k, Tf in enumerate(fine):
                i = int(np.argmin(np.abs(temps - Tf)))
                sums, _ = fss.reweight_sums(series[i][:, 0], series[i][:, 1], d, 1.0 / temps[i],
                                            1.0 / Tf, B)
                e, _, r = fss.jackknife(sums, L * L)
                est[k] = e[0]
                rep[:, k] = r
            curves[L] = (est, rep)
    finally:
        oracle.set_threads(saved)
    t, u, et, eu = fss.crossing_jackknife(fine, curves[8][0], curves[16][0], curves[8][1],
                                          curves[16][1])
    assert not math.isnan(t) and not math.isnan(et)
    assert abs(t - physics.TC_EXACT) < 0.03 + 4 * et
    assert 0.55 < u < 0.68
