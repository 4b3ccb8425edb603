"""Autotuner: it measures and installs a shape, and every tile shape gives
bit-identical results (spins and per-sweep E/M)."""
import numpy as np
import pytest

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
    ising.tuning_clear()


@pytest.mark.parametrize("L", [1024, 2056, 16384])
def test_every_shape_is_bit_identical(I, L):
    I.tuning_clear()
    ref = I.Lattice(L, seed=3, stream_id=1, init=workloads.INIT_HOT, beta=1 / 2.3)
    ref_em = ref.sweep_em(6).cpu().numpy()
    ref_s = ref.get_spins()
    for rpw in (1, 2, 4):
        for mb in (512, 2048):
            I.tuning_set([{"L_min": L, "L_max": L, "rpw": rpw, "max_blocks": mb,
                           "small_lds_bytes": 0, "updates_per_ns": 0.0}])
            lat = I.Lattice(L, seed=3, stream_id=1, init=workloads.INIT_HOT, beta=1 / 2.3)
            assert np.array_equal(lat.sweep_em(6).cpu().numpy(), ref_em), (rpw, mb)
            assert np.array_equal(lat.get_spins(), ref_s), (rpw, mb)
    I.tuning_clear()


def test_autotune_installs_an_entry(I):
    I.tuning_clear()
    e = I.autotune(4096, trial_sweeps=4)
    assert e["L_min"] == 4096 and e["L_max"] == 8191
    assert e["rpw"] in (0, 1, 2, 4) and 1 <= e["max_blocks"] <= 2048
    assert e["updates_per_ns"] > 0
    assert I.tuning_get() == [e]
    small = I.autotune(64, trial_sweeps=20)
    assert small["L_min"] == 64
    I.tuning_clear()
