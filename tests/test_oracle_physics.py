"""Pins the oracle's dynamics to exact statistical mechanics (CPU only).

* 4 x 4 periodic lattice: the exact density of states from enumerating all
  2^16 states is itself pinned to Kaufman's closed-form partition function;
  long oracle runs must reproduce the exact <E>, <M^2>, <M^4>, U4 and the
  exact energy distribution.  A wrong threshold (e.g. exp(-8/T) for dE = 4),
  a wrong neighbour, a wrong colour order or a biased uniform all move these
  averages by many standard errors.
* 32 x 32: Kaufman's exact finite-lattice energy.
* 256 x 256: Onsager's energy and Yang's spontaneous magnetisation.
* Binder cumulant (Eq. (2)) of L = 8 and L = 16 cross between T = 2.20 and
  T = 2.34, bracketing T_c = 2/ln(1+sqrt 2) (the paper quotes 2.269185).
"""
import math

import numpy as np
import pytest

import oracle
import physics


def _series(L, T, n, discard, init_kind=2, seed=1, sid=0, threads=1):
    before = oracle.get_threads()
    oracle.set_threads(threads)
    try:
        s = oracle.init(L, seed, sid, init_kind)
        oracle.sweeps(s, 1.0 / T, seed, sid, 0, discard, record=False)
        EM = oracle.sweeps(s, 1.0 / T, seed, sid, discard, n)
    finally:
        oracle.set_threads(before)
    return EM


def test_enumeration_matches_kaufman():
    dos = physics.density_of_states(4)
    assert sum(dos.values()) == 2 ** 16
    assert dos[-32] == 2 and dos[32] == 2
    assert all(dos[e] == dos[-e] for e in dos)
    E = np.array(list(dos.keys()), dtype=np.float64)
    g = np.array(list(dos.values()), dtype=np.float64)
    for T in (1.7, 2.269185, 3.0, 5.0):
        lz = math.log((g * np.exp(-(E + 32) / T)).sum()) + 32 / T
        assert abs(lz - float(physics.kaufman_logZ(4, 1 / T))) < 1e-10


def test_kaufman_energy_matches_enumeration():
    for T in (2.0, 2.269185, 3.0):
        assert abs(physics.kaufman_energy_per_site(4, T) - physics.exact_moments(4, T)["e"]) < 1e-12


@pytest.mark.parametrize("T", [2.0, 2.269185, 3.0])
def test_4x4_moments_and_energy_distribution(T):
    ex = physics.exact_moments(4, T)
    n = 400_000
    EM = _series(4, T, n, 1000, seed=int(T * 1000))
    N = 16
    E = EM[:, 0].astype(np.float64)
    M = EM[:, 1].astype(np.float64)
    for key, series in (("e", E / N), ("m2", (M / N) ** 2), ("m4", (M / N) ** 4)):
        mean, err = physics.binned_mean_err(series, 100)
        assert abs(mean - ex[key]) < 5 * err + 1e-12, (key, mean, ex[key], err)
    # chi-square of the energy histogram against the exact distribution,
    # using blocks of 20 sweeps to thin the correlations
    thin = EM[::20, 0]
    levels = sorted(ex["p_energy"])
    counts = np.array([(thin == e).sum() for e in levels], dtype=np.float64)
    expect = np.array([ex["p_energy"][e] for e in levels]) * len(thin)
    keep = expect > 20
    chi2 = float((((counts - expect) ** 2) / expect)[keep].sum())
    dof = int(keep.sum()) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)


@pytest.mark.parametrize("T", [2.0, 3.0])
def test_32x32_energy_matches_kaufman(T):
    EM = _series(32, T, 40_000, 2000, threads=4)
    mean, err = physics.binned_mean_err(EM[:, 0] / 1024.0, 50)
    exact = physics.kaufman_energy_per_site(32, T)
    assert abs(mean - exact) < 5 * err, (mean, exact, err)


@pytest.mark.parametrize("T,init_kind", [(2.0, 0), (1.5, 0), (3.0, 2)])
def test_256_matches_onsager(T, init_kind):
    L = 256
    EM = _series(L, T, 1500, 500, init_kind=init_kind, threads=8)
    N = L * L
    e, e_err = physics.binned_mean_err(EM[:, 0] / N, 30)
    assert abs(e - physics.onsager_energy_per_site(T)) < 5 * e_err + 2e-4
    if T < physics.TC_EXACT:
        m, m_err = physics.binned_mean_err(np.abs(EM[:, 1]) / N, 30)
        assert abs(m - physics.spontaneous_magnetisation(T)) < 5 * m_err + 2e-4


def test_binder_cumulants_cross_near_tc():
    U = {}
    for L in (8, 16):
        for T in (2.20, 2.34):
            EM = _series(L, T, 200_000, 2000, seed=L * 100 + int(T * 100))
            U[(L, T)] = physics.binder(EM[:, 1])
    # below T_c the larger lattice is more ordered (U closer to 2/3), above
    # T_c it is less ordered: the curves cross in between.
    assert U[(16, 2.20)] > U[(8, 2.20)]
    assert U[(16, 2.34)] < U[(8, 2.34)]
    assert 0.45 < U[(8, 2.34)] < 2 / 3 and 0.45 < U[(16, 2.20)] < 2 / 3
