"""Light-cone windows of the alternative dynamics (the paper's per-thread
LCG of section 5.3 and its Boltzmann-pattern pools of sections 4 and 5.1).

oracle.lcg_window / oracle.pool_window simulate only a patch around the
window, keyed by global coordinates (generator seeds by the word's global
thread index, pool addresses by the global word index and the sweep), with
a margin of 2n + 1 sites.  They must equal the same window of the
whole-lattice oracle (lcg_sweeps / pool_sweeps, themselves pinned by the
physics tests) bit for bit: at the periodic corners and edges, across a
partial last word (L / 2 not a multiple of 64), from both starts and a later
sweep counter.  A wrong seed index, a draw consumed in the wrong order,
a word skipped when none of its sites is in the patch, or a missed wrap
each fails one of these cases.
"""
import numpy as np
import pytest

import oracle
import workloads

SPOTS = [(0, 0), (-20, -5), (60, 70), (-1, 3), (5, -2), (-64, 40)]


def _cut(s, x0, y0, w, h):
    L = s.shape[0]
    return np.take(np.take(s, np.arange(y0, y0 + h) % L, axis=0), np.arange(x0, x0 + w) % L,
                   axis=1)


@pytest.mark.parametrize("L", [136, 256, 264])
@pytest.mark.parametrize("init", [workloads.INIT_HOT, workloads.INIT_COLD_UP])
@pytest.mark.parametrize("T", [2.269185, 1.5, float("inf")])
def test_lcg_window_equals_the_whole_lattice(L, init, T):
    seed, sid, n = 11, 2, 3
    beta = 0.0 if T == float("inf") else 1.0 / T
    s = oracle.init(L, seed, sid, init)
    st = oracle.lcg_seed(L, seed)
    oracle.lcg_sweeps(s, beta, st, n, record=False)
    for (x0, y0) in SPOTS:
        x0, y0 = x0 % L, y0 % L
        got = oracle.lcg_window(L, beta, seed, sid, init, n, x0, y0, 40, 12)
        assert np.array_equal(got, _cut(s, x0, y0, 40, 12)), (L, init, T, x0, y0)


@pytest.mark.parametrize("L", [136, 264])
@pytest.mark.parametrize("linear", [False, True])
@pytest.mark.parametrize("t0", [0, 5])
def test_pool_window_equals_the_whole_lattice(L, linear, t0):
    seed, sid, n, m = 11, 2, 3, 8
    beta = 1.0 / 2.269185
    pool = oracle.pool_fill(beta, seed, sid, m)
    for init in (workloads.INIT_HOT, workloads.INIT_COLD_DOWN):
        s = oracle.init(L, seed, sid, init)
        oracle.pool_sweeps(s, beta, seed, sid, t0, n, m, linear, record=False)
        for (x0, y0) in SPOTS:
            x0, y0 = x0 % L, y0 % L
            got = oracle.pool_window(L, beta, seed, sid, init, t0, n, m, linear, x0, y0, 40, 12,
                                     pool=pool)
            assert np.array_equal(got, _cut(s, x0, y0, 40, 12)), (L, linear, t0, init, x0, y0)


def test_windows_see_the_dynamics():
    """The windows are not trivially equal: one more sweep of the whole
    lattice changes them, and the LCG and pool windows differ from the
    Philox one."""
    L, seed, sid, n, beta = 136, 11, 2, 2, 1.0 / 2.269185
    s = oracle.init(L, seed, sid, workloads.INIT_HOT)
    st = oracle.lcg_seed(L, seed)
    oracle.lcg_sweeps(s, beta, st, n + 1, record=False)
    lw = oracle.lcg_window(L, beta, seed, sid, workloads.INIT_HOT, n, 10, 10, 40, 12)
    assert not np.array_equal(lw, _cut(s, 10, 10, 40, 12))
    pw = oracle.pool_window(L, beta, seed, sid, workloads.INIT_HOT, 0, n, 8, False, 10, 10, 40,
                            12)
    ph = oracle.window(L, beta, seed, sid, workloads.INIT_HOT, 0, n, 10, 10, 40, 12)
    assert not np.array_equal(lw, ph) and not np.array_equal(pw, ph)


def test_window_size_errors():
    with pytest.raises(ValueError):
        oracle.lcg_window(16, 0.4, 1, 0, workloads.INIT_HOT, 3, 0, 0, 10, 4)  # 10 + 14 > 16
    with pytest.raises(ValueError):
        oracle.pool_window(16, 0.4, 1, 0, workloads.INIT_HOT, 0, 3, 4, False, 0, 0, 4, 10)


def _bands(fn, L, rows):
    total = None
    for y0 in range(0, L, rows):
        em = fn(y0, min(rows, L - y0))
        total = em if total is None else total + em
    return total


@pytest.mark.parametrize("L,rows", [(136, 40), (264, 64), (256, 256 - 2 * 7)])
@pytest.mark.parametrize("init", [workloads.INIT_HOT, workloads.INIT_COLD_DOWN])
def test_lcg_bands_sum_to_the_whole_lattice(L, rows, init):
    """Band sums of (E, M) with light-cone margins equal the whole-lattice
    LCG oracle's per-sweep (E, M) (ragged and aligned L, a band of all but
    the margins, and bands across the periodic wrap)."""
    seed, sid, n, beta = 11, 2, 3, 1.0 / 2.269185
    s = oracle.init(L, seed, sid, init)
    want = oracle.lcg_sweeps(s, beta, oracle.lcg_seed(L, seed), n)
    got = _bands(lambda y0, h: oracle.lcg_band_em(L, beta, seed, sid, init, n, y0, h), L, rows)
    assert np.array_equal(got, want)
    # a band that wraps: rows L - 20 .. L + 19 plus the rest
    wrap = (oracle.lcg_band_em(L, beta, seed, sid, init, n, L - 20, 40) +
            oracle.lcg_band_em(L, beta, seed, sid, init, n, 20, L - 40))
    assert np.array_equal(wrap, want)


@pytest.mark.parametrize("L,rows", [(136, 40), (264, 64)])
@pytest.mark.parametrize("linear", [False, True])
def test_pool_bands_sum_to_the_whole_lattice(L, rows, linear):
    seed, sid, n, m, beta, t0 = 11, 2, 3, 8, 1.0 / 2.269185, 4
    pool = oracle.pool_fill(beta, seed, sid, m)
    for init in (workloads.INIT_HOT, workloads.INIT_COLD_UP):
        s = oracle.init(L, seed, sid, init)
        want = oracle.pool_sweeps(s, beta, seed, sid, t0, n, m, linear)
        got = _bands(lambda y0, h: oracle.pool_band_em(L, beta, seed, sid, init, t0, n, m, linear,
                                                       y0, h, pool=pool), L, rows)
        assert np.array_equal(got, want), (init,)
