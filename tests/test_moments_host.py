"""Exact moment sums of an (E, M) series (ising_series_moments, host code of
the library, the sums a served request reports for the Binder cumulant of
Eq. (2)): sum M^2 and sum M^4 over the kept sweeps, each the exact integer
sum rounded once to the nearest double.  Checked against Python integers,
whose conversion to float is correctly rounded, at magnitudes up to the
largest lattice (|M| = 2^42, so M^4 sums pass 2^128), and on sums placed
exactly halfway between two doubles, where a sum rounded twice or with a
lost low bit goes the wrong way."""
import random

import numpy as np
import pytest


@pytest.fixture(scope="module")
def I():
    from paper_1007_3726_amd import ising
    ising.lib()
    return ising


def _series(ms):
    s = np.zeros((len(ms), 2), dtype=np.int64)
    s[:, 1] = ms
    s[:, 0] = -4 * np.arange(len(ms))  # E plays no part
    return s


def _want(ms, discard):
    kept = [int(m) for m in ms[discard:]]
    return float(sum(m * m for m in kept)), float(sum(m ** 4 for m in kept)), len(kept)


@pytest.mark.parametrize("bits", [4, 20, 31, 36, 42])
def test_random_series(I, bits):
    rng = random.Random(bits)
    lim = 1 << bits
    ms = [rng.randint(-lim, lim) for _ in range(3000)]
    for discard in (0, 7, 2999, 3000, 4000):
        assert I.series_moments(_series(ms), discard) == _want(ms, min(discard, len(ms)))


def test_extremes(I):
    top = 1 << 42
    ms = [top, -top] * 500 + [0, 1, -1]
    assert I.series_moments(_series(ms)) == _want(ms, 0)
    assert float(sum(m ** 4 for m in ms)) > 2.0 ** 128


@pytest.mark.parametrize("big,small,count", [(1 << 25, 1 << 11, 8), (1 << 42, 1 << 28, 8)])
def test_halfway_sums_round_to_even(I, big, small, count):
    # big^4 + count * small^4 = big^4 (1 + 2^-53): exactly halfway, so it
    # rounds down to the even neighbour; one more unit tips it up
    assert big ** 4 + count * small ** 4 == big ** 4 + (big ** 4 >> 53)
    ms = [big] + [small] * count
    _, m4, _ = I.series_moments(_series(ms))
    assert m4 == float(big ** 4)
    _, m4_up, _ = I.series_moments(_series(ms + [1]))
    assert m4_up == float(big ** 4 + count * small ** 4 + 1) > float(big ** 4)


def test_empty_and_errors(I):
    assert I.series_moments(np.zeros((0, 2), dtype=np.int64)) == (0.0, 0.0, 0)
    with pytest.raises(I.IsingError):
        I.series_moments(_series([(1 << 42) + 1]))
    with pytest.raises(I.IsingError):
        I.series_moments(_series([1, 2]), -1)
