"""The Boltzmann-pattern-pool dynamics (section 4's exp4/exp8 pool, the
"unmodified" and "linear" GPU variants of Table 2) on the GPU against the
oracle's pool mode: bit-exact spins and per-sweep int64 (E, M) on ragged
lattices (partial last words, one-word rows, W = 3 and 65), at several
temperatures including beta = 0 and +inf, pool sizes 2^10 .. 2^16, the
pool drawn again when beta changes, lattices past one 256-word group per
row block; argument checks."""
import math
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
    from paper_1007_3726_amd import ising
    ising.lib()
    return ising


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("linear", [False, True])
@pytest.mark.parametrize("L", [8, 16, 24, 64, 136, 200, 264])
@pytest.mark.parametrize("beta", [1 / 2.269185, 0.0, math.inf, 1 / 1.5])
def test_every_sweep_bit_exact(I, L, beta, linear):
    n, m, seed, sid = 6, 10, 7, 3
    _say("case L=%d beta=%r linear=%s" % (L, beta, linear))
    lat = I.Lattice(L, seed=seed, stream_id=sid, init=workloads.INIT_HOT, beta=beta)
    lat.use_pool(m, linear)
    s = oracle.init(L, seed, sid, workloads.INIT_HOT)
    for t in range(n):
        em = lat.sweep_em(1).cpu().numpy()
        oem = oracle.pool_sweeps(s, beta, seed, sid, t, 1, m, linear)
        assert np.array_equal(em, oem), t
        assert np.array_equal(lat.get_spins(), s), t


@pytest.mark.parametrize("L,m,linear", [(1024, 16, True), (1024, 12, False), (2056, 14, True),
                                        (8320, 16, False), (8320, 16, True)])
def test_larger_lattices(I, L, m, linear):
    n, beta = 3, 1 / 2.3
    _say("case L=%d m=%d linear=%s" % (L, m, linear))
    lat = I.Lattice(L, seed=5, init=workloads.INIT_HOT, beta=beta)
    lat.use_pool(m, linear)
    em = lat.sweep_em(n).cpu().numpy()
    s = oracle.init(L, 5, 0, workloads.INIT_HOT)
    oem = oracle.pool_sweeps(s, beta, 5, 0, 0, n, m, linear)
    assert np.array_equal(em, oem)
    assert np.array_equal(lat.get_spins(), s)


@pytest.mark.parametrize("linear", [False, True])
def test_pool_is_drawn_again_when_beta_changes(I, linear):
    L, m = 136, 12
    lat = I.Lattice(L, seed=2, init=workloads.INIT_HOT, beta=0.3)
    lat.use_pool(m, linear)
    s = oracle.init(L, 2, 0, workloads.INIT_HOT)
    e1 = lat.sweep_em(3).cpu().numpy()
    o1 = oracle.pool_sweeps(s, 0.3, 2, 0, 0, 3, m, linear)
    lat.set_beta(0.6)
    e2 = lat.sweep_em(3).cpu().numpy()
    o2 = oracle.pool_sweeps(s, 0.6, 2, 0, 3, 3, m, linear)
    assert np.array_equal(e1, o1) and np.array_equal(e2, o2)
    assert np.array_equal(lat.get_spins(), s)


def test_switching_dynamics(I):
    L, beta = 64, 0.4
    a = I.Lattice(L, seed=2, init=workloads.INIT_HOT, beta=beta)
    ref = a.sweep_em(4).cpu().numpy()
    b = I.Lattice(L, seed=2, init=workloads.INIT_HOT, beta=beta)
    b.use_pool(10)
    b.use_lcg()
    b.use_pool(10, True)
    b.use_philox()
    assert np.array_equal(b.sweep_em(4).cpu().numpy(), ref)


def test_argument_checks(I):
    import torch
    assert I.ising_pool_bytes(10) == 16 << 10 and I.ising_pool_bytes(9) == 0
    assert I.ising_pool_bytes(28) == 16 << 28 and I.ising_pool_bytes(29) == 0
    lat = I.Lattice(66, init=workloads.INIT_HOT, beta=0.4)  # L % 8 != 0
    buf = torch.empty(I.ising_pool_bytes(10), dtype=torch.uint8, device="cuda")
    with pytest.raises(I.IsingError):
        I.check(I.lib().ising_set_rng(lat.h, I.ISING_RNG_POOL, buf.data_ptr(), buf.numel()))
    lat2 = I.Lattice(64, init=workloads.INIT_HOT, beta=0.4)
    with pytest.raises(I.IsingError):  # not 16 * 2^m bytes
        I.check(I.lib().ising_set_rng(lat2.h, I.ISING_RNG_POOL, buf.data_ptr(), 3 << 12))
    with pytest.raises(I.IsingError):  # misaligned
        I.check(I.lib().ising_set_rng(lat2.h, I.ISING_RNG_POOL, buf.data_ptr() + 8, 16 << 10))
    with pytest.raises(I.IsingError):
        I.check(I.lib().ising_set_rng(lat2.h, I.ISING_RNG_POOL_LINEAR, None, 16 << 10))
    lat2.use_pool(10)
    EM = torch.empty((2, 2), dtype=torch.int64, device="cuda")
    with pytest.raises(I.IsingError):
        I.multi_sweep([lat2], 2, [EM])  # batched path: Philox only


@pytest.mark.parametrize("linear", [False, True])
def test_without_series_and_from_a_set_counter(I, linear):
    L, beta, m, t0 = 136, 1 / 2.269185, 11, (1 << 32) - 9
    lat = I.Lattice(L, seed=4, stream_id=2, init=workloads.INIT_HOT, beta=beta)
    lat.use_pool(m, linear)
    lat.sweep_count = t0
    lat.sweep(5)  # no (E, M) series
    em = lat.sweep_em(3).cpu().numpy()
    s = oracle.init(L, 4, 2, workloads.INIT_HOT)
    oracle.pool_sweeps(s, beta, 4, 2, t0, 5, m, linear, record=False)
    oem = oracle.pool_sweeps(s, beta, 4, 2, t0 + 5, 3, m, linear)
    assert np.array_equal(em, oem)
    assert np.array_equal(lat.get_spins(), s)
    assert lat.measure() == (int(oem[-1, 0]), int(oem[-1, 1]))
    with pytest.raises(I.IsingError):  # the counter would pass 2^32 - 1
        lat.sweep(2)


@pytest.mark.parametrize("linear", [False, True])
def test_benchmark_workload(I, linear):
    """16384^2 from a cold start at T = 2.269185 with the benchmark's pool of
    2^22 patterns, both address rules: two sweeps, whole lattice and series."""
    w = workloads.LARGE
    n, m = 2, 22
    _say("case %s pool m=%d linear=%s" % (w.name, m, linear))
    lat = I.Lattice(w.L, seed=w.seed, stream_id=w.stream_id, init=w.init, beta=1.0 / w.T)
    lat.use_pool(m, linear)
    em = lat.sweep_em(n).cpu().numpy()
    s = oracle.init(w.L, w.seed, w.stream_id, w.init)
    oem = oracle.pool_sweeps(s, 1.0 / w.T, w.seed, w.stream_id, 0, n, m, linear)
    assert np.array_equal(em, oem)
    assert np.array_equal(lat.get_spins(), s)


def _alt_golden(L, T, seed, sid, init, dyn):
    """{sweep: (E, M)} of tests/golden/alt_em.txt (the oracle's band sums)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "alt_em.txt")
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if (int(f[0]), float(f[1]), int(f[2]), int(f[3]), int(f[4]), f[5]) == (L, T, seed, sid,
                                                                             init, dyn):
            out[int(f[6])] = (int(f[7]), int(f[8]))
    return out


SPOTS = [(0, 0), (-20, -5), (-7, 100), (123456, -3), (0.5, 0.5), (-64, 777)]


@pytest.mark.parametrize("linear", [False, True])
@pytest.mark.parametrize("L,T,n", [(262144, 2.0, 3), (100008, 2.269185, 2)])
def test_large_lattices_in_light_cone_windows(I, L, T, n, linear):
    """The HBM-resident 262144^2 lattice (where the pool kernels are
    profiled) and 100008^2 (782 words per row, the last one partial) with the
    benchmark's pool of 2^22 patterns, both address rules, from a hot start:
    windows at the periodic corners, edges and centre equal the oracle's
    light-cone windows of the same dynamics; every (E, M) obeys the
    invariants and the last equals a recount."""
    import torch
    seed, m = 7, 22
    beta = 1.0 / T
    _say("case L=%d pool m=%d linear=%s, %d sweeps" % (L, m, linear, n))
    lat = I.Lattice(L, seed=seed, stream_id=0, init=workloads.INIT_HOT, beta=beta)
    lat.use_pool(m, linear)
    EM = lat.sweep_em(n).cpu().numpy()
    N = L * L
    assert np.all(EM[:, 0] % 4 == 0) and np.all((EM[:, 1] - N) % 2 == 0)
    assert np.all(np.abs(EM[:, 0]) <= 2 * N) and np.all(np.abs(EM[:, 1]) <= N)
    assert lat.measure() == (int(EM[-1, 0]), int(EM[-1, 1]))
    gold = _alt_golden(L, T, seed, 0, workloads.INIT_HOT, "pool22-linear" if linear else "pool22")
    if L == 262144:
        assert sorted(gold) == list(range(1, n + 1)), "no oracle values for this case"
    for k, (e, mm) in gold.items():
        assert (int(EM[k - 1, 0]), int(EM[k - 1, 1])) == (e, mm), k
    pool = oracle.pool_fill(beta, seed, 0, m)
    for (sx, sy) in SPOTS:
        x0 = int(sx * L) % L if isinstance(sx, float) else sx % L
        y0 = int(sy * L) % L if isinstance(sy, float) else sy % L
        got = lat.get_window(x0, y0, 40, 12)
        want = oracle.pool_window(L, beta, seed, 0, workloads.INIT_HOT, 0, n, m, linear, x0, y0,
                                  40, 12, pool=pool)
        assert np.array_equal(got, want), (L, linear, x0, y0)
    del lat
    torch.cuda.empty_cache()


def _large_alt(dyn):
    """(E/M rows [2000, 2], {sweep: sha256}) of tests/golden/large_alt_*.txt."""
    here = os.path.dirname(os.path.abspath(__file__))
    em, sha = [], {}
    for line in open(os.path.join(here, "golden", "large_alt_em.txt")):
        f = line.split()
        if f and not f[0].startswith("#") and f[0] == dyn:
            em.append((int(f[2]), int(f[3])))
    for line in open(os.path.join(here, "golden", "large_alt_sha256.txt")):
        f = line.split()
        if f and not f[0].startswith("#") and f[0] == dyn:
            sha[int(f[1])] = f[2]
    return np.array(em, dtype=np.int64), sha


def test_benchmark_workload_all_sweeps(I):
    """16384^2 from a cold start at T = 2.269185 with the benchmark's pool of
    2^22 patterns at random addresses, all 2000 sweeps the benchmark times per
    step: every (E, M) and the spin array at sweeps 1, 10 and 2000 (sha256)
    against the oracle's stored values (tests/golden/make_large_alt.py)."""
    import hashlib
    ref_em, ref_sha = _large_alt("pool22")
    w = workloads.LARGE
    assert len(ref_em) == w.sweeps and sorted(ref_sha) == [1, 10, w.sweeps]
    _say("case %s pool22, %d sweeps" % (w.name, w.sweeps))
    lat = I.Lattice(w.L, seed=w.seed, stream_id=w.stream_id, init=w.init, beta=1.0 / w.T)
    lat.use_pool(22, False)
    done, ems = 0, []
    for t in sorted(ref_sha):
        ems.append(lat.sweep_em(t - done).cpu().numpy())
        done = t
        d = hashlib.sha256(np.ascontiguousarray(lat.get_spins()).tobytes()).hexdigest()
        assert d == ref_sha[t], "spins differ after sweep %d" % t
    assert np.array_equal(np.concatenate(ems, axis=0), ref_em)
