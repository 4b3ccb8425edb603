"""The per-thread-LCG dynamics (the paper's own random numbers) on the GPU
against the oracle's LCG mode: bit-exact spins, per-sweep int64 (E, M) and
generator states, on ragged lattices (partial last words, one-word rows,
W = 65), at several temperatures including beta = 0 and +inf; seeding;
checkpoint/resume of spins and states; argument checks."""
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


def _lcg_lattice(I, L, seed, init, beta):
    lat = I.Lattice(L, seed=seed, stream_id=0, init=init, beta=beta)
    lat.use_lcg()
    return lat


@pytest.mark.parametrize("L", [8, 16, 24, 64, 136, 200])
@pytest.mark.parametrize("beta", [1 / 2.269185, 0.0, math.inf, 1 / 1.5])
def test_every_sweep_bit_exact(I, L, beta):
    n = 10
    _say("case L=%d beta=%r" % (L, beta))
    lat = _lcg_lattice(I, L, 7, workloads.INIT_HOT, beta)
    assert np.array_equal(lat.lcg_states(), oracle.lcg_seed(L, 7))
    s = oracle.init(L, 7, 0, workloads.INIT_HOT)
    st = oracle.lcg_seed(L, 7)
    for t in range(n):
        em = lat.sweep_em(1).cpu().numpy()
        oem = oracle.lcg_sweeps(s, beta, st, 1)
        assert np.array_equal(em, oem), t
        assert np.array_equal(lat.get_spins(), s), t
    assert np.array_equal(lat.lcg_states(), st)


@pytest.mark.parametrize("L,seed,init", [(1024, 3, workloads.INIT_HOT),
                                         (2056, 12345, workloads.INIT_COLD_UP),
                                         (8320, 1, workloads.INIT_HOT)])
def test_larger_lattices(I, L, seed, init):
    n = 3
    beta = 1 / 2.3
    _say("case L=%d" % L)
    lat = _lcg_lattice(I, L, seed, init, beta)
    em = lat.sweep_em(n).cpu().numpy()
    s = oracle.init(L, seed, 0, init)
    st = oracle.lcg_seed(L, seed)
    oem = oracle.lcg_sweeps(s, beta, st, n)
    assert np.array_equal(em, oem)
    assert np.array_equal(lat.get_spins(), s)
    assert np.array_equal(lat.lcg_states(), st)


def test_checkpoint_and_resume(I):
    import torch
    L, beta = 136, 0.42
    a = _lcg_lattice(I, L, 4, workloads.INIT_HOT, beta)
    a.sweep(12)
    full = a.get_spins()
    b = _lcg_lattice(I, L, 4, workloads.INIT_HOT, beta)
    b.sweep(5)
    spins, states = b.get_spins(), b.lcg_states().copy()
    c = _lcg_lattice(I, L, 99, workloads.INIT_COLD_DOWN, beta)
    c.set_spins(spins)
    c.lcg_buf.copy_(torch.from_numpy(states.view(np.int32).reshape(-1)).view(torch.uint8).cuda())
    c.sweep(7)
    assert np.array_equal(c.get_spins(), full)


def test_philox_and_lcg_switch(I):
    L, beta = 64, 0.4
    a = I.Lattice(L, seed=2, init=workloads.INIT_HOT, beta=beta)
    ref = a.sweep_em(4).cpu().numpy()
    b = I.Lattice(L, seed=2, init=workloads.INIT_HOT, beta=beta)
    b.use_lcg()
    b.use_philox()
    assert np.array_equal(b.sweep_em(4).cpu().numpy(), ref)


def test_argument_checks(I):
    import torch
    lat = I.Lattice(66, init=workloads.INIT_HOT, beta=0.4)  # L % 8 != 0
    buf = torch.empty(I.ising_lcg_bytes(66), dtype=torch.uint8, device="cuda")
    with pytest.raises(I.IsingError):
        I.check(I.lib().ising_set_rng(lat.h, I.ISING_RNG_LCG, buf.data_ptr(), buf.numel()))
    lat2 = I.Lattice(64, init=workloads.INIT_HOT, beta=0.4)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(I.IsingError) as e:
        I.check(I.lib().ising_set_rng(lat2.h, I.ISING_RNG_LCG, small.data_ptr(), 16))
    assert e.value.code == I.ISING_ENOMEM
    with pytest.raises(I.IsingError):
        I.check(I.lib().ising_set_rng(lat2.h, 7, None, 0))
    lat2.use_lcg()
    EM = torch.empty((2, 2), dtype=torch.int64, device="cuda")
    with pytest.raises(I.IsingError):
        I.multi_sweep([lat2], 2, [EM])  # batched path is Philox only
    assert I.ising_lcg_bytes(64) == 2 * 64 * 1 * 4 and I.ising_lcg_bytes(7) == 0


def test_benchmark_workload(I):
    """16384^2 from a cold start at T = 2.269185, seed 1, as the benchmark
    runs it: two sweeps, whole lattice, series and generator states."""
    w = workloads.LARGE
    n = 2
    _say("case %s lcg, %d sweeps" % (w.name, n))
    lat = _lcg_lattice(I, w.L, w.seed, w.init, 1.0 / w.T)
    em = lat.sweep_em(n).cpu().numpy()
    s = oracle.init(w.L, w.seed, w.stream_id, w.init)
    st = oracle.lcg_seed(w.L, w.seed)
    oem = oracle.lcg_sweeps(s, 1.0 / w.T, st, n)
    assert np.array_equal(em, oem)
    assert np.array_equal(lat.get_spins(), s)
    assert np.array_equal(lat.lcg_states(), st)


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


@pytest.mark.parametrize("L,T,n", [(262144, 2.0, 3), (100008, 2.269185, 2)])
def test_large_lattices_in_light_cone_windows(I, L, T, n):
    """The HBM-resident 262144^2 lattice (where the LCG kernel is profiled)
    and 100008^2 (782 words per row, the last one partial) with the LCG
    dynamics from a hot start: windows at the periodic corners, edges and
    centre equal the oracle's light-cone windows of the same dynamics; every
    (E, M) obeys the invariants and the last equals a recount."""
    import torch
    seed = 7
    _say("case L=%d lcg, %d sweeps" % (L, n))
    lat = _lcg_lattice(I, L, seed, workloads.INIT_HOT, 1.0 / T)
    EM = lat.sweep_em(n).cpu().numpy()
    N = L * L
    assert np.all(EM[:, 0] % 4 == 0) and np.all((EM[:, 1] - N) % 2 == 0)
    assert np.all(np.abs(EM[:, 0]) <= 2 * N) and np.all(np.abs(EM[:, 1]) <= N)
    assert lat.measure() == (int(EM[-1, 0]), int(EM[-1, 1]))
    gold = _alt_golden(L, T, seed, 0, workloads.INIT_HOT, "lcg")
    if L == 262144:
        assert sorted(gold) == list(range(1, n + 1)), "no oracle values for this case"
    for k, (e, mm) in gold.items():
        assert (int(EM[k - 1, 0]), int(EM[k - 1, 1])) == (e, mm), k
    for (sx, sy) in SPOTS:
        x0 = int(sx * L) % L if isinstance(sx, float) else sx % L
        y0 = int(sy * L) % L if isinstance(sy, float) else sy % L
        got = lat.get_window(x0, y0, 40, 12)
        want = oracle.lcg_window(L, 1.0 / T, seed, 0, workloads.INIT_HOT, n, x0, y0, 40, 12)
        assert np.array_equal(got, want), (L, x0, y0)
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
    """16384^2 from a cold start at T = 2.269185 with the LCG dynamics, all
    2000 sweeps the benchmark times per step: every (E, M) and the spin array
    at sweeps 1, 10 and 2000 (sha256) against the oracle's stored values
    (tests/golden/make_large_alt.py)."""
    import hashlib
    ref_em, ref_sha = _large_alt("lcg")
    w = workloads.LARGE
    assert len(ref_em) == w.sweeps and sorted(ref_sha) == [1, 10, w.sweeps]
    _say("case %s lcg, %d sweeps" % (w.name, w.sweeps))
    lat = _lcg_lattice(I, w.L, w.seed, w.init, 1.0 / w.T)
    done, ems = 0, []
    for t in sorted(ref_sha):
        ems.append(lat.sweep_em(t - done).cpu().numpy())
        done = t
        d = hashlib.sha256(np.ascontiguousarray(lat.get_spins()).tobytes()).hexdigest()
        assert d == ref_sha[t], "spins differ after sweep %d" % t
    assert np.array_equal(np.concatenate(ems, axis=0), ref_em)
