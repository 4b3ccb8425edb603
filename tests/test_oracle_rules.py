"""Pins the oracle's update rule, thresholds and invariants (CPU only).

Each check is against something fixed outside the oracle: the Eq. (5)
bit-pattern form of the acceptance rule with the exp4/exp8 encoding of
section 4, high-precision arithmetic for the thresholds, symmetries of the
Hamiltonian (Eq. (1)), and the exact binomial law of the first colour step
from an ordered start.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle

TEMPS = [2.269, 2.269185, 2.0, 3.0, 1.5, 3.5, 2.2, 2.34]


def _exact_threshold(beta, dE):
    with mpmath.workdps(60):
        v = mpmath.floor(mpmath.exp(-mpmath.mpf(beta) * dE) * mpmath.mpf(2) ** 32)
        return int(min(v, 2 ** 32 - 1))


@pytest.mark.parametrize("T", TEMPS)
def test_thresholds_match_high_precision(T):
    beta = 1.0 / T
    t4, t8 = oracle.thresholds(beta)
    assert (t4, t8) == (_exact_threshold(beta, 4), _exact_threshold(beta, 8))
    assert 0 < t8 < t4 < 2 ** 32


def test_threshold_edges():
    assert oracle.thresholds(0.0) == (2 ** 32 - 1, 2 ** 32 - 1)
    assert oracle.thresholds(math.inf) == (0, 0)
    for bad in (-1e-9, -1.0, math.nan, -math.inf):
        with pytest.raises(ValueError):
            oracle.thresholds(bad)


def test_acceptance_truth_table():
    # Eq. (5): i1+i2+i3+i4 + 2*exp8 + exp4 >= 2 with i_n = s0 ^ s_n (Eq. (4)),
    # exp8 = [r < e^-8/T], exp4 = [e^-8/T <= r < e^-4/T]  (section 4),
    # i.e. 2*exp8 + exp4 = [u < t4] + [u < t8].
    for T in (2.269185, 1.5, 3.5):
        t4, t8 = oracle.thresholds(1.0 / T)
        us = sorted({0, t8 - 1, t8, t8 + 1, t4 - 1, t4, t4 + 1, 2 ** 32 - 1})
        for pattern in range(32):
            bits = [(pattern >> b) & 1 for b in range(5)]
            s0, ns = bits[0], bits[1:]
            k = sum(s0 ^ n for n in ns)
            for u in us:
                eq5 = int(k + int(u < t4) + int(u < t8) >= 2)
                spin = lambda b: 1 if b else -1
                got = oracle.accept(spin(s0), *[spin(n) for n in ns], u, t4, t8)
                assert got == eq5, (T, pattern, u)


def test_hot_start_uses_phase_2_and_3():
    L = 64
    s = oracle.init(L, 9, 4, 2)
    for (x, y) in [(0, 0), (1, 0), (5, 9), (63, 63), (10, 33)]:
        u = oracle.uniform(9, 4, 2 + ((x + y) & 1), 0, L, x, y)
        assert s[y, x] == (1 if u < 2 ** 31 else -1)
    frac = (s == 1).mean()
    assert abs(frac - 0.5) < 5 * 0.5 / L


@pytest.mark.parametrize("L", [4, 6, 10, 34])
def test_invariants_along_a_run(L):
    s, EM = oracle.run(L, 1 / 2.269185, 3, 1, 2, 300)
    N = L * L
    E, M = EM[:, 0], EM[:, 1]
    assert np.all(E % 4 == 0)
    assert np.all((M - N) % 2 == 0)
    assert np.all(np.abs(E) <= 2 * N) and np.all(np.abs(M) <= N)
    assert not np.any(E == -2 * N + 4)
    assert (int(E[-1]), int(M[-1])) == oracle.measure(s)


def test_ordered_states_energy():
    for L in (4, 8, 10):
        assert oracle.measure(np.ones((L, L), np.int8)) == (-2 * L * L, L * L)
        cb = np.fromfunction(lambda y, x: 1 - 2 * ((x + y) % 2), (L, L)).astype(np.int8)
        assert oracle.measure(cb) == (2 * L * L, 0)


@pytest.mark.parametrize("L", [6, 16, 34])
def test_global_flip_mirror(L):
    # The rule depends only on s0 ^ s_n and the uniforms, so the all -1 start
    # must give exactly the negated trajectory of the all +1 start.
    sp, EMp = oracle.run(L, 1 / 2.269, 21, 2, 0, 50)
    sm, EMm = oracle.run(L, 1 / 2.269, 21, 2, 1, 50)
    assert np.array_equal(sm, -sp)
    assert np.array_equal(EMm[:, 0], EMp[:, 0])
    assert np.array_equal(EMm[:, 1], -EMp[:, 1])


def test_zero_temperature_quench():
    # beta = +inf: t4 = t8 = 0, only dE <= 0 moves; E never increases.
    L = 32
    s, EM = oracle.run(L, math.inf, 5, 0, 2, 40)
    E0, _ = oracle.measure(oracle.init(L, 5, 0, 2))
    E = [E0] + list(EM[:, 0])
    assert all(b <= a for a, b in zip(E, E[1:]))


def test_first_colour_step_is_binomial():
    # From all +1 every colour-0 site has k = 0 (dE = 8), so the number of
    # flipped colour-0 sites after one sweep is Binomial(n, t8 / 2^32).
    L, T = 128, 2.269185
    t4, t8 = oracle.thresholds(1 / T)
    p = t8 / 2 ** 32
    total = 0
    n = 0
    for seed in range(12):
        s = oracle.init(L, seed, 0, 0)
        oracle.sweeps(s, 1 / T, seed, 0, 0, 1, record=False)
        c0 = (np.add.outer(np.arange(L), np.arange(L)) % 2) == 0
        total += int((s[c0] == -1).sum())
        n += int(c0.sum())
    mean, sd = n * p, math.sqrt(n * p * (1 - p))
    assert abs(total - mean) < 5 * sd


@pytest.mark.parametrize("x0,y0", [(0, 0), (60, 3), (27, 61), (40, 40)])
def test_light_cone_window_matches_full_lattice(x0, y0):
    L, n, w, h = 64, 6, 9, 7
    beta = 1 / 2.269
    s, _ = oracle.run(L, beta, 77, 3, 2, n)
    win = oracle.window(L, beta, 77, 3, 2, 0, n, x0, y0, w, h)
    ys = [(y0 + j) % L for j in range(h)]
    xs = [(x0 + i) % L for i in range(w)]
    assert np.array_equal(win, s[np.ix_(ys, xs)])
