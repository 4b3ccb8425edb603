"""The strict Metropolis compare of Eq. (3) on the device, at its boundary.

For a colour-0 site of a hot-start lattice, the oracle's Philox gives the
uniform u the site draws at sweep 0.  beta is then chosen so that the
site's threshold is exactly u + 1 (u < t: the flip is accepted) or exactly
u (rejected): t4 for a site with one anti-aligned neighbour (Delta E = 4),
t8 for a site with none (Delta E = 8).  The device must flip the site in the
first case only, and its whole lattice after one sweep must equal the
oracle's.  An off-by-one compare (<= for <) or swapped thresholds on the
device fails here on a single site, where the statistical tests could not
see it.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def I():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1007_3726_amd import ising
    ising.lib()
    return ising


def _beta_for(target: int, dE: int) -> float:
    """A beta with floor(exp(-dE beta) 2^32) == target (oracle thresholds)."""
    idx = 0 if dE == 4 else 1
    b = -math.log((target + 0.5) / 2.0 ** 32) / dE
    lo, hi = b * (1 - 1e-6), b * (1 + 1e-6)  # t(lo) >= target >= t(hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        t = oracle.thresholds(mid)[idx]
        if t == target:
            return mid
        if t > target:
            lo = mid
        else:
            hi = mid
    raise AssertionError("no beta gives threshold %d" % target)


def _anti(s, x, y):
    L = s.shape[0]
    c = s[y, x]
    return sum(int(s[yy % L, xx % L] != c)
               for xx, yy in ((x - 1, y), (x + 1, y), (x, y - 1), (x, y + 1)))


def _site(s0, seed, sid, k):
    """First colour-0 site with k anti-aligned neighbours, and its uniform."""
    L = s0.shape[0]
    for y in range(L):
        for x in range(L):
            if (x + y) % 2 == 0 and _anti(s0, x, y) == k:
                u = oracle.uniform(seed, sid, 0, 0, L, x, y)
                if 1 <= u <= 2 ** 32 - 2:
                    return x, y, u
    raise AssertionError("no site with k = %d" % k)


@pytest.mark.parametrize("seed", [3, 17, 40])
@pytest.mark.parametrize("k,dE", [(1, 4), (0, 8)])
def test_threshold_boundary_on_the_device(I, seed, k, dE):
    L, sid = 16, 5
    s0 = oracle.init(L, seed, sid, workloads.INIT_HOT)
    x, y, u = _site(s0, seed, sid, k)
    for t, flips in ((u + 1, True), (u, False)):
        beta = _beta_for(t, dE)
        print("case seed=%d k=%d t=%d flips=%s beta=%r" % (seed, k, t, flips, beta), flush=True)
        sys.stdout.flush()
        want, _ = oracle.run(L, beta, seed, sid, workloads.INIT_HOT, 1)
        assert (want[y, x] != s0[y, x]) == flips  # the oracle's own strict compare
        lat = I.Lattice(L, seed=seed, stream_id=sid, init=workloads.INIT_HOT, beta=beta)
        assert tuple(lat.thresholds()) == oracle.thresholds(beta)
        assert lat.thresholds()[0 if dE == 4 else 1] == t
        lat.sweep(1)
        got = lat.get_spins()
        assert (got[y, x] != s0[y, x]) == flips
        assert np.array_equal(got, want)


@pytest.mark.parametrize("seed", [3, 17, 40])
def test_each_class_uses_its_own_threshold(I, seed):
    """A site with no anti-aligned neighbour at t4 = u + 1 (so t8 < u) must
    stay; a site with one at t8 = u (so t4 > u) must flip.  A device that
    compared Delta E = 8 sites with t4, or Delta E = 4 sites with t8, fails."""
    L, sid = 16, 5
    s0 = oracle.init(L, seed, sid, workloads.INIT_HOT)
    for k, t_of, dE, flips in ((0, 1, 4, False), (1, 0, 8, True)):
        x, y, u = _site(s0, seed, sid, k)
        beta = _beta_for(u + t_of, dE)
        t4, t8 = oracle.thresholds(beta)
        assert (t8 < u < t4) if k == 0 else (t8 == u < t4)
        print("case seed=%d k=%d t4=%d t8=%d u=%d" % (seed, k, t4, t8, u), flush=True)
        want, _ = oracle.run(L, beta, seed, sid, workloads.INIT_HOT, 1)
        assert (want[y, x] != s0[y, x]) == flips
        lat = I.Lattice(L, seed=seed, stream_id=sid, init=workloads.INIT_HOT, beta=beta)
        assert tuple(lat.thresholds()) == (t4, t8)
        lat.sweep(1)
        got = lat.get_spins()
        assert (got[y, x] != s0[y, x]) == flips
        assert np.array_equal(got, want)
