"""Pins the oracle's band-by-band (E, M) against its whole-lattice run (CPU only).

``oracle.band_em`` computes one band of rows' shares of the energy (Eq. (1),
each bond counted at its left or upper end) and of the magnetisation after
each sweep, simulating only the band and a light-cone margin of 2n + 1 rows
on each side.  Summed over bands that partition the rows it must give the
whole-lattice series of ``oracle.run`` exactly; each band alone must equal
the same rows' shares recomputed from the whole-lattice spins.  A margin one
row too small, a bond counted at the wrong end, a band keyed by band-local
instead of global rows, or a missed periodic wrap in x fails these checks.
"""
import numpy as np
import pytest

import oracle

INIT_COLD_UP, INIT_COLD_DOWN, INIT_HOT = 0, 1, 2


def _row_shares(s):
    """Per-row (E, M) shares of an int8 L x L configuration (numpy, int64)."""
    v = s.astype(np.int64)
    e = -(v * (np.roll(v, -1, axis=1) + np.roll(v, -1, axis=0))).sum(axis=1)
    return e, v.sum(axis=1)


def _whole(L, T, seed, sid, init_kind, n):
    """Whole-lattice spins after every sweep and the per-sweep (E, M)."""
    s = oracle.init(L, seed, sid, init_kind)
    states, EM = [], []
    for t in range(n):
        EM.append(oracle.sweeps(s, 1.0 / T, seed, sid, t, 1)[0])
        states.append(s.copy())
    return states, np.array(EM)


@pytest.mark.parametrize("L,T,init_kind,n,band", [
    (16, 2.269185, INIT_HOT, 2, 4),
    (34, 2.0, INIT_HOT, 3, 7),        # band height does not divide L
    (20, 3.0, INIT_COLD_UP, 2, 5),
    (12, 1.5, INIT_COLD_DOWN, 1, 3),
    (130, 2.269185, INIT_HOT, 4, 33),  # W = 2 words per colour row, partial last word
    (64, 5.0, INIT_HOT, 3, 64 - 14),   # one band as large as the margin allows, then the rest
])
def test_bands_sum_to_the_whole_lattice(L, T, init_kind, n, band):
    seed, sid = 1234 + L, 5
    states, EM = _whole(L, T, seed, sid, init_kind, n)
    got = oracle.lattice_em_by_bands(L, 1.0 / T, seed, sid, init_kind, n, band)
    assert np.array_equal(got, EM)
    # and every band alone equals the same rows of the whole-lattice state
    y0 = 0
    while y0 < L:
        h = min(band, L - y0)
        part = oracle.band_em(L, 1.0 / T, seed, sid, init_kind, 0, n, y0, h)
        for k in range(n):
            e, m = _row_shares(states[k])
            assert part[k, 0] == e[y0:y0 + h].sum() and part[k, 1] == m[y0:y0 + h].sum()
        y0 += h


def test_band_across_the_periodic_wrap():
    """A band whose margin wraps from the last rows to the first."""
    L, T, n = 40, 2.269185, 3
    states, _ = _whole(L, T, 99, 0, INIT_HOT, n)
    for y0, h in ((0, 5), (L - 3, 3), (L - 12, 12)):
        part = oracle.band_em(L, 1.0 / T, 99, 0, INIT_HOT, 0, n, y0, h)
        for k in range(n):
            e, m = _row_shares(states[k])
            rows = [(y0 + j) % L for j in range(h)]
            assert part[k, 0] == e[rows].sum() and part[k, 1] == m[rows].sum()


def test_band_from_a_later_sweep_counter():
    """t0 > 0: the uniforms of sweep t0 + k, from a fresh start (as oracle_window)."""
    L, T, n, t0 = 24, 2.269185, 2, 17
    s = oracle.init(L, 3, 1, INIT_HOT)
    EM = oracle.sweeps(s, 1.0 / T, 3, 1, t0, n)
    tot = np.zeros((n, 2), dtype=np.int64)
    for y0 in range(0, L, 6):
        tot += oracle.band_em(L, 1.0 / T, 3, 1, INIT_HOT, t0, n, y0, 6)
    assert np.array_equal(tot, EM)


def test_zero_temperature_quench_and_high_temperature():
    """beta = +inf (RNG-free) and beta = 0 (every move accepted but with prob 2^-32)."""
    L, n = 28, 3
    for beta in (float("inf"), 0.0):
        s = oracle.init(L, 8, 0, INIT_HOT)
        EM = oracle.sweeps(s, beta, 8, 0, 0, n)
        got = oracle.lattice_em_by_bands(L, beta, 8, 0, INIT_HOT, n, 8)
        assert np.array_equal(got, EM)


def test_size_errors():
    with pytest.raises(ValueError):
        oracle.band_em(16, 0.5, 1, 0, INIT_HOT, 0, 3, 0, 4)   # 4 + 2 * 7 > 16
    with pytest.raises(ValueError):
        oracle.band_em(16, 0.5, 1, 0, INIT_HOT, 0, 1, 0, 0)
