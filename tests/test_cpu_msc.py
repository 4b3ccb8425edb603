"""The multi-spin-coded CPU baseline (``baselines/msc_cpu.c``) against the
oracle: the same Markov chain bit for bit (spins after every sweep and the
per-sweep E/M) on aligned and ragged lattices, every start, temperatures
including beta = 0 and +inf, with the AVX-512 and the scalar Philox and
with 1 and 4 threads; the vector Philox's carry into the counter's high word
against the oracle's uniforms site by site."""
import math

import numpy as np
import pytest

import baselines
import oracle
import workloads

BETAS = [1 / 2.269185, 0.0, math.inf, 1 / 1.5]


@pytest.fixture(params=["vector", "scalar"])
def path(request):
    if request.param == "vector" and not baselines.vector_available():
        pytest.skip("no AVX-512 on this CPU")
    baselines.scalar_only(request.param == "scalar")
    yield request.param
    baselines.scalar_only(False)


@pytest.mark.parametrize("L", [4, 8, 10, 64, 66, 130, 136, 200])
@pytest.mark.parametrize("init", [workloads.INIT_COLD_UP, workloads.INIT_COLD_DOWN,
                                  workloads.INIT_HOT])
def test_every_sweep_equals_the_oracle(path, L, init):
    seed, sid = 12345, 3
    b = baselines.Lattice(L, seed=seed, stream_id=sid, init=init, threads=1)
    s = oracle.init(L, seed, sid, init)
    assert np.array_equal(b.spins(), s)
    t = 0
    for beta in BETAS:
        for _ in range(2):
            em = b.sweeps(beta, 1)
            oem = oracle.sweeps(s, beta, seed, sid, t, 1)
            t += 1
            assert np.array_equal(em, oem), (beta, t)
            assert np.array_equal(b.spins(), s), (beta, t)


@pytest.mark.parametrize("L", [1024, 1000])
def test_threads_and_a_larger_lattice(path, L):
    beta = 1 / 2.3
    a = baselines.Lattice(L, seed=9, init=workloads.INIT_HOT, threads=1)
    b = baselines.Lattice(L, seed=9, init=workloads.INIT_HOT, threads=4)
    ea, eb = a.sweeps(beta, 3), b.sweeps(beta, 3)
    s, oem = oracle.run(L, beta, 9, 0, workloads.INIT_HOT, 3)
    assert np.array_equal(ea, oem) and np.array_equal(eb, oem)
    assert np.array_equal(a.spins(), s) and np.array_equal(b.spins(), s)


def test_vector_philox_carries_into_the_high_counter_word():
    if not baselines.vector_available():
        pytest.skip("no AVX-512 on this CPU")
    L, seed, sid, t = 185368, 77, 5, 9
    L8, W = L // 8, (L // 2 + 63) // 64
    # words whose 16 Philox blocks straddle 2^32: lo32(g0) > 2^32 - 16
    found = []
    for y in range(L):
        rem = (1 << 32) - y * L8  # 16 w must lie in [rem - 15, rem - 1]
        if rem <= 0:
            break
        w = (rem - 1) // 16
        if w < W and 16 * w >= rem - 15:
            found.append((y, w))
    assert found
    ta, tb = 0x9000_0000, 0x2000_0000
    for (y, w) in found:
        for phase in (0, 1):
            got = baselines.word_masks(L, seed, sid, y, w, t, phase, ta, tb)
            want = [0, 0]
            for b in range(64):
                k = 64 * w + b
                x = 2 * k + ((y + phase) & 1)
                u = oracle.uniform(seed, sid, phase, t, L, x, y)
                want[0] |= (u < ta) << b
                want[1] |= (u < tb) << b
            assert got == tuple(want), (y, w, phase)


def test_argument_checks():
    with pytest.raises(ValueError):
        baselines.Lattice(7)
    b = baselines.Lattice(8)
    with pytest.raises(ValueError):
        b.sweeps(-1.0, 1)
    with pytest.raises(ValueError):
        b.sweeps(float("nan"), 1)


@pytest.mark.parametrize("linear", [False, True])
@pytest.mark.parametrize("L,m", [(8, 10), (24, 12), (136, 12), (200, 14), (1024, 16)])
def test_pool_dynamics_equal_the_oracle(path, L, m, linear):
    beta, seed, sid = 1 / 2.269185, 9, 2
    b = baselines.Lattice(L, seed=seed, stream_id=sid, init=workloads.INIT_HOT, threads=2)
    b.use_pool(beta, m, linear)
    s = oracle.init(L, seed, sid, workloads.INIT_HOT)
    for t in range(3):
        em = b.pool_sweeps(1)
        oem = oracle.pool_sweeps(s, beta, seed, sid, t, 1, m, linear)
        assert np.array_equal(em, oem), t
        assert np.array_equal(b.spins(), s), t
