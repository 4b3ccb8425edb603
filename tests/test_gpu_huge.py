"""Lattices too large for the byte-per-spin oracle to hold.

262144 x 262144 (8 GiB packed, HBM-resident), hot start from seed 7, at
T = 2.0 and 3.0 for the benchmark's 100 sweeps; 1048576^2 (2^33 words per
colour plane) and 185368^2 (more than 2^32 Philox blocks per colour, L not a
power of two).

* The per-sweep int64 (E, M) is compared bit for bit with the oracle's
  whole-lattice values (tests/golden/huge_em.txt, written by
  tests/golden/make_huge_em.py from the oracle alone, which sums the
  lattice band by band with light-cone margins): sweeps 1-10 at 262144^2,
  1-4 at 185368^2 and sweep 1 at 1048576^2.
* Spins are checked with light-cone windows: after n sweeps a site depends
  only on initial spins and uniforms within Manhattan distance 2n, so the
  oracle simulates a (w + 4n + 2)^2 patch keyed by global coordinates whose
  inner w x h window must equal the GPU's, bit for bit.  Windows sit at the
  corners (periodic wrap in both directions), edges and centre.
* Every sweep's (E, M) obeys the invariants of any configuration, and the
  last one equals an independent recount of the final state.
"""
import os
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
    if torch.cuda.get_device_properties(0).total_memory < 16 * (1 << 30):
        pytest.skip("needs > 16 GiB of device memory")
    from paper_1007_3726_amd import ising
    ising.lib()
    return ising


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _golden():
    """{(L, T, seed, stream_id, init): {sweep: (E, M)}} from the oracle's file."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "huge_em.txt")
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        key = (int(f[0]), float(f[1]), int(f[2]), int(f[3]), int(f[4]))
        out.setdefault(key, {})[int(f[5])] = (int(f[6]), int(f[7]))
    return out


GOLDEN = _golden()


def _check_golden(key, EM, required):
    ref = GOLDEN.get(key)
    if ref is None:
        assert not required, "no oracle values for %r" % (key,)
        _say("  (no oracle E/M for %r yet)" % (key,))
        return
    for k, (e, m) in sorted(ref.items()):
        if k <= len(EM):
            assert (int(EM[k - 1, 0]), int(EM[k - 1, 1])) == (e, m), "sweep %d of %r" % (k, key)
    _say("  E/M of sweeps %s equal the oracle's" % sorted(ref))


@pytest.mark.parametrize("w", [workloads.HUGE_T2, workloads.HUGE_T3])
def test_huge_lattice_windows(I, w):
    L, n = w.L, w.sweeps
    _say("case %s: %d sweeps" % (w.name, n))
    lat = I.Lattice(L, seed=w.seed, stream_id=w.stream_id, init=w.init, beta=1.0 / w.T)
    EM = lat.sweep_em(n).cpu().numpy()
    _check_golden((L, w.T, w.seed, w.stream_id, w.init), EM, required=True)
    N = L * L
    assert np.all(EM[:, 0] % 4 == 0) and np.all((EM[:, 1] - N) % 2 == 0)
    assert np.all(np.abs(EM[:, 0]) <= 2 * N) and np.all(np.abs(EM[:, 1]) <= N)
    assert lat.measure() == (int(EM[-1, 0]), int(EM[-1, 1]))
    # energy per site relaxes towards the infinite-lattice value
    e = EM[-1, 0] / N
    assert -2.0 <= e <= -0.5
    ww, hh = 40, 12
    spots = [(0, 0), (L - 20, L - 5), (L - 7, 100), (123456, L - 3), (L // 2, L // 2),
             (131000, 77)]
    for (x0, y0) in spots:
        got = lat.get_window(x0, y0, ww, hh)
        ref = oracle.window(L, 1.0 / w.T, w.seed, w.stream_id, w.init, 0, n, x0, y0, ww, hh)
        assert np.array_equal(got, ref), "window at (%d, %d) differs" % (x0, y0)
    del lat


def _windows_and_invariants(I, L, T, seed, n, spots):
    lat = I.Lattice(L, seed=seed, stream_id=0, init=workloads.INIT_HOT, beta=1.0 / T)
    EM = lat.sweep_em(n).cpu().numpy()
    _check_golden((L, T, seed, 0, workloads.INIT_HOT), EM, required=True)
    N = L * L
    assert np.all(EM[:, 0] % 4 == 0) and np.all((EM[:, 1] - N) % 2 == 0)
    assert np.all(np.abs(EM[:, 0]) <= 2 * N) and np.all(np.abs(EM[:, 1]) <= N)
    assert lat.measure() == (int(EM[-1, 0]), int(EM[-1, 1]))
    ww, hh = 40, 12
    for (x0, y0) in spots:
        got = lat.get_window(x0, y0, ww, hh)
        ref = oracle.window(L, 1.0 / T, seed, 0, workloads.INIT_HOT, 0, n, x0, y0, ww, hh)
        assert np.array_equal(got, ref), "window at (%d, %d) differs" % (x0, y0)
    del lat


def test_largest_lattice_that_fits(I):
    """1048576^2 (128 GiB packed): each colour plane holds 2^33 words, so
    word indices, tile counts and per-block bond counts pass 32 bits, and
    Philox block indices reach 2^37."""
    import torch
    if torch.cuda.get_device_properties(0).total_memory < 160 * (1 << 30):
        pytest.skip("needs > 160 GiB of device memory")
    L = 1 << 20
    assert L * (L // 128) >= 1 << 32
    _say("case L=%d" % L)
    spots = [(0, 0), (L - 20, L - 5), (L - 7, 1000), (777777, L - 3), (L // 2, L // 2)]
    _windows_and_invariants(I, L, 2.0, 7, 3, spots)
    torch.cuda.empty_cache()


def test_non_power_of_two_past_2_to_the_32_blocks(I):
    """185368^2: more than 2^32 Philox blocks per colour and L not a power
    of two, so rows straddle a change of the counter's high word (the
    general colour-step kernel serves this shape)."""
    import torch
    L = 185368
    assert L % 8 == 0 and L * L // 8 > 1 << 32 and L & (L - 1)
    _say("case L=%d" % L)
    # the first row whose block indices straddle 2^32: y L/8 < 2^32 < (y+1) L/8
    ys = (1 << 32) // (L // 8)
    spots = [(0, 0), (L - 20, L - 5), (L - 30, ys - 4), (5000, ys - 2), (L // 2, L // 2)]
    _windows_and_invariants(I, L, 2.269185, 11, 4, spots)
    torch.cuda.empty_cache()
