"""Autotuner: it measures and installs a shape, and every tile and strip
shape gives bit-identical results (spins and per-sweep E/M), and the
default shape's run equals the oracle's (whole lattice up to 10008^2,
light-cone windows above)."""
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
    ising.tuning_clear()


def _against_oracle(em, spins, L, beta, seed, sid, init):
    """The default shape's run (the reference every other shape is held
    to) against the oracle: the whole lattice up to 10008^2, light-cone
    windows at the corners, an edge and the centre above."""
    n = len(em)
    if L <= 10008:
        s, oem = oracle.run(L, beta, seed, sid, init, n)
        assert np.array_equal(em, oem)
        assert np.array_equal(spins, s)
        return
    for (x0, y0) in [(0, 0), (L - 20, L - 5), (L - 7, 1000), (L // 2, L // 2)]:
        want = oracle.window(L, beta, seed, sid, init, 0, n, x0, y0, 40, 12)
        got = np.take(np.take(spins, np.arange(y0, y0 + 12) % L, axis=0),
                      np.arange(x0, x0 + 40) % L, axis=1)
        assert np.array_equal(got, want), (x0, y0)


@pytest.mark.parametrize("L", [1024, 2056, 16384])
def test_every_shape_is_bit_identical(I, L):
    I.tuning_clear()
    ref = I.Lattice(L, seed=3, stream_id=1, init=workloads.INIT_HOT, beta=1 / 2.3)
    ref_em = ref.sweep_em(6).cpu().numpy()
    ref_s = ref.get_spins()
    _against_oracle(ref_em, ref_s, L, 1 / 2.3, 3, 1, workloads.INIT_HOT)
    for rpw in (1, 2, 4):
        for mb in (512, 2048):
            I.tuning_set([{"L_min": L, "L_max": L, "form": I.ISING_FORM_TILE, "rpw": rpw,
                           "max_blocks": mb, "small_lds_bytes": 0, "updates_per_ns": 0.0}])
            lat = I.Lattice(L, seed=3, stream_id=1, init=workloads.INIT_HOT, beta=1 / 2.3)
            assert np.array_equal(lat.sweep_em(6).cpu().numpy(), ref_em), (rpw, mb)
            assert np.array_equal(lat.get_spins(), ref_s), (rpw, mb)
    I.tuning_clear()


# W = 63 (one partial segment), 65 (a one-word second segment), 79 with a
# partial last word (12 valid bits), and 128 full words
@pytest.mark.parametrize("L", [8000, 8320, 10008, 16384])
def test_strip_shapes_match_tiles(I, L):
    I.tuning_clear()
    ref = I.Lattice(L, seed=5, stream_id=3, init=workloads.INIT_HOT, beta=1 / 2.25)
    ref_em = ref.sweep_em(5).cpu().numpy()
    ref_s = ref.get_spins()
    _against_oracle(ref_em, ref_s, L, 1 / 2.25, 5, 3, workloads.INIT_HOT)
    # rows per task: the size rule, tails of 1..3 rows after the 4-row
    # unrolled cycle, and tasks longer than one resident wave's share
    for rows in (0, 1, 3, 4, 7, 64):
        for mb in (512, 2048):
            I.tuning_set([{"L_min": L, "L_max": L, "form": I.ISING_FORM_STRIP, "rpw": rows,
                           "max_blocks": mb, "small_lds_bytes": 0, "updates_per_ns": 0.0}])
            lat = I.Lattice(L, seed=5, stream_id=3, init=workloads.INIT_HOT, beta=1 / 2.25)
            assert np.array_equal(lat.sweep_em(5).cpu().numpy(), ref_em), (rows, mb)
            assert np.array_equal(lat.get_spins(), ref_s), (rows, mb)
    I.tuning_clear()


def test_strip_form_falls_back_to_tiles_for_narrow_rows(I):
    # W = 8 words per row: the strip form does not apply and tiles run
    L = 1024
    I.tuning_clear()
    ref = I.Lattice(L, seed=2, init=workloads.INIT_HOT, beta=0.44)
    ref_em = ref.sweep_em(4).cpu().numpy()
    I.tuning_set([{"L_min": L, "L_max": L, "form": I.ISING_FORM_STRIP, "rpw": 4,
                   "max_blocks": 2048, "small_lds_bytes": 0, "updates_per_ns": 0.0}])
    lat = I.Lattice(L, seed=2, init=workloads.INIT_HOT, beta=0.44)
    assert np.array_equal(lat.sweep_em(4).cpu().numpy(), ref_em)
    I.tuning_clear()


def test_autotune_installs_an_entry(I):
    I.tuning_clear()
    e = I.autotune(4096, trial_sweeps=4)
    assert e["L_min"] == 4096 and e["L_max"] == 8191
    assert e["form"] in (I.ISING_FORM_TILE, I.ISING_FORM_STRIP)
    assert 0 <= e["rpw"] <= 4096 and 1 <= e["max_blocks"] <= 2048
    assert e["updates_per_ns"] > 0
    assert I.tuning_get() == [e]
    small = I.autotune(64, trial_sweeps=20)
    assert small["L_min"] == 64
    I.tuning_clear()
