"""Pins of the oracle's per-thread-LCG dynamics (the paper's own random
numbers, section 5.3, Eqs. (6) and (7)).

* thread seeds equal seed * 16807^j mod 2^32 (Python's modular power, not
  the oracle's recurrence);
* after n sweeps every thread's state is its seed advanced 64 n times,
  computed here by an affine jump-ahead (doubling of the map x -> a x + c)
  rather than by stepping;
* from a cold start, the colour-0 sites that flip in the first sweep are
  exactly those whose LCG value (site 63 of each word first) has
  |int32(x)| < t8', predicted here site by site;
* thresholds equal floor(exp(-beta dE) 2^31) in 60-digit arithmetic;
* at beta = +inf the LCG and Philox dynamics give the same (deterministic)
  trajectory;
* the 4 x 4 lattice samples the exact distribution (enumeration) at
  T = 2.269185 and 3.0, and a 32 x 32 lattice Kaufman's exact energy.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
import physics
import workloads

A, C, MOD = 1664525, 1013904223, 1 << 32


def jump(x, n):
    """The affine map x -> A x + C applied n times, by doubling."""
    mul, add = 1, 0            # accumulated map: x -> mul x + add
    pm, pa = A, C              # map for the current power of two
    while n:
        if n & 1:
            mul, add = (pm * mul) % MOD, (pm * add + pa) % MOD
        pm, pa = (pm * pm) % MOD, (pm * pa + pa) % MOD
        n >>= 1
    return (mul * x + add) % MOD


@pytest.mark.parametrize("L,seed", [(8, 1), (136, 12345), (64, (7 << 40) | 99)])
def test_seeds_are_powers_of_16807(L, seed):
    st = oracle.lcg_seed(L, seed).ravel()
    s0 = seed & 0xFFFFFFFF
    for j in list(range(min(20, len(st)))) + [len(st) - 1, len(st) // 2, 12345 % len(st)]:
        assert int(st[j]) == (s0 * pow(16807, j, MOD)) % MOD, j
    if seed == 1:
        assert list(st[:3]) == [1, 16807, 282475249]  # Eq. (7) with x_{0,0} = 1


@pytest.mark.parametrize("L", [8, 24, 136])
def test_states_advance_64_per_sweep(L):
    st0 = oracle.lcg_seed(L, 5)
    st = st0.copy()
    s = oracle.init(L, 5, 0, workloads.INIT_HOT)
    n = 3
    oracle.lcg_sweeps(s, 0.4, st, n, record=False)
    want = np.array([jump(int(x), 64 * n) for x in st0.ravel()], dtype=np.uint32)
    assert np.array_equal(st.ravel(), want)


@pytest.mark.parametrize("L,beta", [(8, 0.3), (24, 0.44), (136, 0.2)])
def test_cold_start_first_colour_step_flips_are_predicted(L, beta):
    s = oracle.init(L, 1, 0, workloads.INIT_COLD_UP)
    st = oracle.lcg_seed(L, 9)
    seeds = st.copy()
    oracle.lcg_sweeps(s, beta, st, 1, record=False)
    t8 = int(mpmath.floor(mpmath.exp(-8 * mpmath.mpf(beta)) * 2 ** 31))
    half = L // 2
    W = (half + 63) // 64
    for y in range(L):
        for w in range(W):
            x = int(seeds[0, y, w])
            for k in range(1, 65):
                x = (A * x + C) % MOD
                site = 64 * w + 64 - k
                if site >= half:
                    continue
                sx = x - MOD if x >= 1 << 31 else x
                px = 2 * site + (y & 1)
                # every colour-0 neighbour is +1 at the first colour-0 step: dE = 8
                assert s[y, px] == (-1 if abs(sx) < t8 else 1), (y, px)


@pytest.mark.parametrize("beta", [0.0, 0.1, 1 / 2.269185, 0.9, 3.0])
def test_thresholds_in_60_digits(beta):
    mpmath.mp.dps = 60
    got = oracle.lcg_thresholds(beta)
    for dE, g in zip((4, 8), got):
        want = min(int(mpmath.floor(mpmath.exp(-dE * mpmath.mpf(beta)) * 2 ** 31)), 1 << 31)
        assert g == want
    assert oracle.lcg_thresholds(math.inf) == (0, 0)


def test_zero_temperature_quench_is_rng_free():
    L = 64
    a = oracle.init(L, 3, 0, workloads.INIT_HOT)
    b = a.copy()
    st = oracle.lcg_seed(L, 3)
    ea = oracle.lcg_sweeps(a, math.inf, st, 20)
    eb = oracle.sweeps(b, math.inf, 3, 0, 0, 20)
    assert np.array_equal(a, b) and np.array_equal(ea, eb)


@pytest.mark.parametrize("T", [2.269185, 3.0])
def test_4x4_samples_the_exact_distribution(T):
    ex = physics.exact_moments(4, T)
    s = oracle.init(4, 11, 0, workloads.INIT_HOT)
    st = oracle.lcg_seed(4, 11)
    saved = oracle.get_threads()
    oracle.set_threads(1)
    try:
        oracle.lcg_sweeps(s, 1.0 / T, st, 1000, record=False)
        EM = oracle.lcg_sweeps(s, 1.0 / T, st, 300_000)
    finally:
        oracle.set_threads(saved)
    E = EM[:, 0].astype(np.float64) / 16
    M = EM[:, 1].astype(np.float64) / 16
    for key, series in (("e", E), ("m2", M ** 2), ("m4", M ** 4)):
        mean, err = physics.binned_mean_err(series, 100)
        assert abs(mean - ex[key]) < 5 * err + 1e-12, (key, mean, ex[key], err)


def test_32x32_energy_matches_kaufman():
    T = 2.0
    s = oracle.init(32, 4, 0, workloads.INIT_COLD_UP)
    st = oracle.lcg_seed(32, 4)
    oracle.lcg_sweeps(s, 1.0 / T, st, 2000, record=False)
    EM = oracle.lcg_sweeps(s, 1.0 / T, st, 40_000)
    mean, err = physics.binned_mean_err(EM[:, 0] / 1024.0, 50)
    assert abs(mean - physics.kaufman_energy_per_site(32, T)) < 5 * err
