"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bit-exact spins and exact int64 (E, M) after every sweep on small and ragged
lattices (partial last words, rows whose Philox blocks straddle rows, the
LDS-resident single-workgroup path and the grid-stride path), all three
initial states, and beta in {0, 1/1.5, 1/2.269, 1/3.5, +inf}.
"""
import hashlib
import math
import os
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


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


def gpu_series(I, L, beta, seed, sid, init, n, per_sweep_spins=False):
    lat = I.Lattice(L, seed=seed, stream_id=sid, init=init, beta=beta)
    spins = [lat.get_spins()]
    ems = []
    if per_sweep_spins:
        for _ in range(n):
            ems.append(lat.sweep_em(1).cpu().numpy())
            spins.append(lat.get_spins())
        EM = np.concatenate(ems, axis=0)
    else:
        EM = lat.sweep_em(n).cpu().numpy()
        spins.append(lat.get_spins())
    return lat, spins, EM


def oracle_series(L, beta, seed, sid, init, n, per_sweep_spins=False):
    s = oracle.init(L, seed, sid, init)
    spins = [s.copy()]
    if per_sweep_spins:
        ems = []
        for t in range(n):
            ems.append(oracle.sweeps(s, beta, seed, sid, t, 1))
            spins.append(s.copy())
        return spins, np.concatenate(ems, axis=0)
    EM = oracle.sweeps(s, beta, seed, sid, 0, n)
    spins.append(s.copy())
    return spins, EM


SMALL_L = [4, 6, 8, 10, 12, 34, 64, 66, 128, 130, 200, 256]
BETAS = [1 / 2.269, 0.0, math.inf, 1 / 1.5, 1 / 3.5]


@pytest.mark.parametrize("L", SMALL_L)
@pytest.mark.parametrize("init", [workloads.INIT_HOT, workloads.INIT_COLD_UP,
                                  workloads.INIT_COLD_DOWN])
def test_every_sweep_bit_exact(I, L, init):
    beta = 1 / 2.269
    n = 12
    _say("case L=%d init=%d n=%d" % (L, init, n))
    lat, gs, gEM = gpu_series(I, L, beta, 3, 5, init, n, per_sweep_spins=True)
    os_, oEM = oracle_series(L, beta, 3, 5, init, n, per_sweep_spins=True)
    assert np.array_equal(gs[0], os_[0]), "initial state differs"
    for t in range(1, n + 1):
        assert np.array_equal(gs[t], os_[t]), "spins differ after sweep %d" % t
    assert np.array_equal(gEM, oEM)
    assert lat.measure() == tuple(int(v) for v in oEM[-1])


@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("L", [6, 64, 130, 384])
def test_temperatures_bit_exact(I, L, beta):
    n = 30
    _say("case L=%d beta=%r n=%d" % (L, beta, n))
    lat, gs, gEM = gpu_series(I, L, beta, 11, 0, workloads.INIT_HOT, n)
    os_, oEM = oracle_series(L, beta, 11, 0, workloads.INIT_HOT, n)
    assert np.array_equal(gEM, oEM)
    assert np.array_equal(gs[-1], os_[-1])
    assert lat.thresholds() == oracle.thresholds(beta)


def test_small_plain_workload(I):
    # 64 x 64, T = 2.269, hot start from seed 1, 1000 sweeps, E/M every sweep.
    w = workloads.SMALL
    _say("case %s" % w.name)
    lat, gs, gEM = gpu_series(I, w.L, 1 / w.T, w.seed, w.stream_id, w.init, w.sweeps)
    os_, oEM = oracle_series(w.L, 1 / w.T, w.seed, w.stream_id, w.init, w.sweeps)
    assert np.array_equal(gEM, oEM)
    assert np.array_equal(gs[-1], os_[-1])


@pytest.mark.parametrize("L", [512, 1024, 1030])
def test_medium_lattices(I, L):
    n = 8
    _say("case L=%d n=%d" % (L, n))
    lat, gs, gEM = gpu_series(I, L, 1 / 2.3, 17, 9, workloads.INIT_HOT, n)
    os_, oEM = oracle_series(L, 1 / 2.3, 17, 9, workloads.INIT_HOT, n)
    assert np.array_equal(gEM, oEM)
    assert np.array_equal(gs[-1], os_[-1])


def test_large_plain_workload_against_stored_oracle(I):
    """16384 x 16384, T = 2.269185, cold start, 2000 sweeps: every (E, M) and
    the full spin array at sweeps 1, 10 and 2000 (sha256) against the
    oracle's stored values (tests/golden/make_large_plain.py)."""
    em_path = os.path.join(HERE, "golden", "large_plain_em.txt")
    sha_path = os.path.join(HERE, "golden", "large_plain_sha256.txt")
    if not (os.path.exists(em_path) and os.path.exists(sha_path)):
        pytest.skip("stored oracle reference not generated")
    ref_em = np.loadtxt(em_path, dtype=np.int64, comments="#")
    ref_sha = {}
    for ln in open(sha_path):
        if ln.startswith("#") or not ln.strip():
            continue
        t, d = ln.split()
        ref_sha[int(t)] = d
    w = workloads.LARGE
    _say("case %s" % w.name)
    lat = I.Lattice(w.L, seed=w.seed, stream_id=w.stream_id, init=w.init, beta=1 / w.T)
    done = 0
    ems = []
    for t in sorted(ref_sha):
        ems.append(lat.sweep_em(t - done).cpu().numpy())
        done = t
        d = hashlib.sha256(np.ascontiguousarray(lat.get_spins()).tobytes()).hexdigest()
        assert d == ref_sha[t], "spins differ after sweep %d" % t
    assert np.array_equal(np.concatenate(ems, axis=0), ref_em)


def test_checkpoint_resume(I):
    L, beta, n, k = 130, 1 / 2.4, 20, 7
    a = I.Lattice(L, seed=4, stream_id=1, init=workloads.INIT_HOT, beta=beta)
    a.sweep(n)
    full = a.get_spins()
    b = I.Lattice(L, seed=4, stream_id=1, init=workloads.INIT_HOT, beta=beta)
    b.sweep(k)
    snap, t = b.get_spins(), b.sweep_count
    c = I.Lattice(L, seed=4, stream_id=1, init=workloads.INIT_COLD_DOWN, beta=beta)
    c.set_spins(snap)
    c.sweep_count = t
    c.sweep(n - k)
    assert np.array_equal(c.get_spins(), full)


def test_mirror_symmetry(I):
    L, beta = 256, 1 / 2.269
    up = I.Lattice(L, seed=8, init=workloads.INIT_COLD_UP, beta=beta)
    dn = I.Lattice(L, seed=8, init=workloads.INIT_COLD_DOWN, beta=beta)
    eu = up.sweep_em(25).cpu().numpy()
    ed = dn.sweep_em(25).cpu().numpy()
    assert np.array_equal(up.get_spins(), -dn.get_spins())
    assert np.array_equal(eu[:, 0], ed[:, 0]) and np.array_equal(eu[:, 1], -ed[:, 1])


def test_set_get_roundtrip_and_windows(I):
    L = 66
    rng = np.random.default_rng(3)
    s = np.where(rng.random((L, L)) < 0.5, 1, -1).astype(np.int8)
    lat = I.Lattice(L, init=workloads.INIT_COLD_UP)
    lat.set_spins(s)
    assert np.array_equal(lat.get_spins(), s)
    win = lat.get_window(60, 50, 10, 20)
    assert np.array_equal(win, s[np.ix_([(50 + j) % L for j in range(20)],
                                        [(60 + i) % L for i in range(10)])])
    assert lat.measure() == oracle.measure(s)
    bad = s.copy()
    bad[3, 4] = 0
    with pytest.raises(I.IsingError):
        lat.set_spins(bad)


def test_error_paths(I):
    lat = I.Lattice(64, init=workloads.INIT_HOT)
    with pytest.raises(I.IsingError):
        lat.sweep(1)  # no beta yet
    for bad in (-1.0, math.nan):
        with pytest.raises(I.IsingError):
            lat.set_beta(bad)
    lat.set_beta(0.4)
    with pytest.raises(I.IsingError):
        lat.sweep(-1)
    lat.sweep_count = 2 ** 32 - 2
    with pytest.raises(I.IsingError):
        lat.sweep(3)
    lat.sweep(2)
    assert lat.sweep_count == 2 ** 32
    lat.sweep(0)


@pytest.mark.parametrize("L", [7936, 8000, 8064, 8192])
def test_rows_of_62_to_64_words(I, L):
    """W = 62, 63, 63, 64 words per row: the narrow/wide tile-shape boundary.
    Full-lattice (E, M) against the oracle for 2 sweeps, and windows that
    include the row seam and the periodic wrap."""
    n = 2
    beta = 1 / 2.4
    _say("case L=%d (W=%d)" % (L, ((L // 2) + 63) // 64))
    lat = I.Lattice(L, seed=13, stream_id=2, init=workloads.INIT_HOT, beta=beta)
    gEM = lat.sweep_em(n).cpu().numpy()
    s, oEM = oracle_series(L, beta, 13, 2, workloads.INIT_HOT, n)
    assert np.array_equal(gEM, oEM)
    for (x0, y0) in [(0, 0), (L - 20, L - 9), (L // 2 - 3, 17)]:
        win = lat.get_window(x0, y0, 24, 12)
        ref = s[-1][np.ix_([(y0 + j) % L for j in range(12)], [(x0 + i) % L for i in range(24)])]
        assert np.array_equal(win, ref)


@pytest.mark.parametrize("L", [8, 16, 24, 32, 64, 128, 136, 200, 256, 264])
def test_lds_resident_lanes_per_word(I, L):
    """The single-workgroup LDS-resident path (forced by a tuning entry): 2-8
    lanes per word for L % 8 == 0 with 128-512 words per plane (128 .. 264),
    one lane per word otherwise: every sweep bit-exact, partial last words
    included (136: 4 valid bits, 200: 36, 264: 4 in the third word)."""
    I.tuning_set([{"L_min": L, "L_max": L, "form": I.ISING_FORM_TILE, "rpw": 0,
                   "max_blocks": 2048, "small_lds_bytes": 65536, "updates_per_ns": 0.0}])
    try:
        beta = 1 / 2.269185
        n = 6
        _say("case LDS-resident L=%d" % L)
        lat, gs, gEM = gpu_series(I, L, beta, 21, 2, workloads.INIT_HOT, n, per_sweep_spins=True)
        os_, oEM = oracle_series(L, beta, 21, 2, workloads.INIT_HOT, n, per_sweep_spins=True)
        assert np.array_equal(gEM, oEM)
        for t in range(n + 1):
            assert np.array_equal(gs[t], os_[t]), t
    finally:
        I.tuning_clear()
