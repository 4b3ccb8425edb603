"""Race test of the kernels that synchronise through block barriers inside a
launch (the LDS-resident small-lattice sweeps and the packed persistent
batched kernel): with the barrier-perturbation hook on, every wave pauses a
pseudo-random time before each barrier, and the spins and per-sweep (E, M)
must stay bit-identical to the unperturbed run and to the oracle."""
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
    yield ising
    ising.debug_perturb(0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("seed", [1, 0xBEEF, 123456789])
@pytest.mark.parametrize("L", [16, 64, 128, 96])
def test_lds_resident_sweeps(I, seed, L):
    n, beta = 8, 1 / 2.269185
    _say("case L=%d seed=%d" % (L, seed))
    I.debug_perturb(seed)
    try:
        lat = I.Lattice(L, seed=3, init=workloads.INIT_HOT, beta=beta)
        em = lat.sweep_em(n).cpu().numpy()
        spins = lat.get_spins()
    finally:
        I.debug_perturb(0)
    s, oem = oracle.run(L, beta, 3, 0, workloads.INIT_HOT, n)
    assert np.array_equal(em, oem)
    assert np.array_equal(spins, s)


@pytest.mark.parametrize("seed", [7, 99])
def test_packed_batched_kernel(I, seed):
    import torch
    Ls = [8, 16, 24, 64, 72, 128, 136, 256]
    n = 6
    _say("case packed seed=%d" % seed)

    def run(perturb):
        lats = [I.Lattice(L, seed=5 + i, stream_id=i, init=workloads.INIT_HOT,
                          beta=1 / (2.1 + 0.05 * i)) for i, L in enumerate(Ls)]
        EMs = [torch.empty((n, 2), dtype=torch.int64, device="cuda") for _ in lats]
        I.debug_perturb(perturb)
        try:
            I.multi_sweep(lats, n, EMs, form="packed")  # packed persistent form
        finally:
            I.debug_perturb(0)
        return [e.cpu().numpy() for e in EMs], [lat.get_spins() for lat in lats]

    e0, s0 = run(0)
    e1, s1 = run(seed)
    for i, L in enumerate(Ls):
        assert np.array_equal(e0[i], e1[i]) and np.array_equal(s0[i], s1[i]), L
        s, oem = oracle.run(L, 1 / (2.1 + 0.05 * i), 5 + i, i, workloads.INIT_HOT, n)
        assert np.array_equal(e1[i], oem) and np.array_equal(s1[i], s), L
