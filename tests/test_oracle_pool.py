"""Pins of the oracle's Boltzmann-pattern-pool dynamics (section 4's pool of
exp4/exp8 patterns, read at a random address per update, or linearly from
one random start per group of 256 words as in the "linear" GPU variant of
Table 2).

* the fraction of set exp8 / exp4 bits is t8 / 2^32 and (t4 - t8) / 2^32
  within binomial errors;
* a few patterns recomputed bit by bit from Philox4x32-10 and the paper's
  encoding (exp8 iff r < e^{-8 beta}, exp4 iff e^{-8 beta} <= r < e^{-4 beta});
* at beta = +inf the pool is empty and the dynamics is the deterministic
  zero-temperature quench of the per-site dynamics;
* at beta = 0 every pattern bit is set, so every spin flips in every colour
  step and one sweep negates the lattice;
* from a cold start the colour-0 sites that flip in the first sweep are
  exactly the exp8 bits of the patterns at the addresses the definition
  gives (random and linear), predicted here word by word;
* a 4 x 4 lattice samples the exact distribution (enumeration) at
  T = 2.269185, in both variants, with a pool of 2^20 patterns.  A finite
  pool is biased: the 4 x 4 lattice reads only bits 0 and 1 of its
  patterns, whose empirical acceptance rates differ from e^{-8 beta} by
  about P^{-1/2} relative (2 % at P = 2^16, which shifts <E>/N by 0.009,
  5.7 of this test's standard errors; 0.5 % at P = 2^20, about 1.4).
"""
import math

import numpy as np
import pytest

import oracle
import physics
import workloads


def _pop(a):
    return sum(bin(int(v)).count("1") for v in a)


@pytest.mark.parametrize("beta", [1 / 2.269185, 1 / 1.5, 1 / 3.5])
def test_bit_fractions(beta):
    m = 14
    e4, e8 = oracle.pool_fill(beta, 3, 1, m)
    t4, t8 = oracle.thresholds(beta)
    n = 64 << m
    for got, p in ((_pop(e8), t8 / 2 ** 32), (_pop(e4), (t4 - t8) / 2 ** 32)):
        sd = math.sqrt(n * p * (1 - p))
        assert abs(got - n * p) < 5 * sd + 1, (got, n * p, sd)
    assert not np.any(e4 & e8)  # the two encodings are exclusive


def test_patterns_bit_by_bit():
    beta, seed, sid, m = 0.41, (5 << 33) | 17, 2, 10
    e4, e8 = oracle.pool_fill(beta, seed, sid, m)
    t4, t8 = oracle.thresholds(beta)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    for p in (0, 1, 517, (1 << m) - 1):
        for b in range(64):
            i = 64 * p + b
            u = oracle.philox4x32_10((i // 4, 0, 0xFFFFFFFF, (sid << 2) | 2), key)[i % 4]
            assert ((int(e8[p]) >> b) & 1) == (u < t8)
            assert ((int(e4[p]) >> b) & 1) == (t8 <= u < t4)


@pytest.mark.parametrize("linear", [False, True])
def test_zero_temperature_quench_is_rng_free(linear):
    L = 64
    a = oracle.init(L, 3, 0, workloads.INIT_HOT)
    b = a.copy()
    ea = oracle.pool_sweeps(a, math.inf, 3, 0, 0, 20, 10, linear)
    eb = oracle.sweeps(b, math.inf, 3, 0, 0, 20)
    assert np.array_equal(a, b) and np.array_equal(ea, eb)


@pytest.mark.parametrize("linear", [False, True])
def test_infinite_temperature_negates_the_lattice(linear):
    L, m = 66, 10
    e4, e8 = oracle.pool_fill(0.0, 4, 0, m)
    assert all(int(v) == (1 << 64) - 1 for v in e8)  # u = 2^32 - 1 was never drawn
    s = oracle.init(L, 4, 0, workloads.INIT_HOT)
    s0 = s.copy()
    oracle.pool_sweeps(s, 0.0, 4, 0, 0, 1, m, linear)
    assert np.array_equal(s, -s0)


@pytest.mark.parametrize("L,linear", [(24, False), (136, False), (1024, True), (200, True)])
def test_cold_start_first_step_is_predicted(L, linear):
    beta, seed, sid, m = 0.3, 9, 1, 12
    e4, e8 = oracle.pool_fill(beta, seed, sid, m)
    s = oracle.init(L, seed, sid, workloads.INIT_COLD_UP)
    oracle.pool_sweeps(s, beta, seed, sid, 0, 1, m, linear, record=False)
    W = (L // 2 + 63) // 64
    key = (seed, 0)
    for y in range(L):
        for w in range(W):
            j = y * W + w
            q = j // 256 if linear else j
            v = oracle.philox4x32_10((q, 0, 0, (sid << 2) | 0), key)[0]
            a = v >> (32 - m)
            if linear:
                a = (a + j % 256) % (1 << m)
            bits = int(e8[a])
            for b in range(min(64, L // 2 - 64 * w)):
                x = 2 * (64 * w + b) + (y & 1)
                # every neighbour is +1 at the first colour-0 step: k = 0
                assert s[y, x] == (-1 if (bits >> b) & 1 else 1), (y, x)


@pytest.mark.parametrize("linear", [False, True])
def test_4x4_samples_the_exact_distribution(linear):
    T = 2.269185
    ex = physics.exact_moments(4, T)
    s = oracle.init(4, 11, 0, workloads.INIT_HOT)
    saved = oracle.get_threads()
    oracle.set_threads(1)
    try:
        oracle.pool_sweeps(s, 1.0 / T, 11, 0, 0, 1000, 20, linear, record=False)
        EM = oracle.pool_sweeps(s, 1.0 / T, 11, 0, 1000, 200_000, 20, linear)
    finally:
        oracle.set_threads(saved)
    E = EM[:, 0].astype(np.float64) / 16
    M = EM[:, 1].astype(np.float64) / 16
    for key, series in (("e", E), ("m2", M ** 2), ("m4", M ** 4)):
        mean, err = physics.binned_mean_err(series, 100)
        assert abs(mean - ex[key]) < 5 * err + 1e-12, (key, mean, ex[key], err)


def test_bad_pool_size():
    s = oracle.init(8, 1, 0, workloads.INIT_HOT)
    with pytest.raises(ValueError):
        oracle.pool_sweeps(s, 0.4, 1, 0, 0, 1, 0, False)
