"""Host-side checks of the batched autotuner's installed shape (no GPU):
set/get/clear and argument validation."""
import ctypes

import pytest


@pytest.fixture(scope="module")
def I():
    from paper_1007_3726_amd import ising
    ising.lib()
    return ising


def test_set_get_clear(I):
    I.batch_tuning_clear()
    d = I.batch_tuning_get()
    assert not d["installed"]
    assert (d["rpw_max"], d["wg_per_cu"], d["graph_chunk"]) == (2, 8, 32)  # built-in
    try:
        I.batch_tuning_set(4, 6, 16)
        d = I.batch_tuning_get()
        assert d["installed"] and (d["rpw_max"], d["wg_per_cu"], d["graph_chunk"]) == (4, 6, 16)
    finally:
        I.batch_tuning_clear()
    assert not I.batch_tuning_get()["installed"]


@pytest.mark.parametrize("shape", [(3, 8, 32), (0, 8, 32), (8, 8, 32), (2, 0, 32), (2, 9, 32),
                                   (2, 8, -1), (2, 8, 4097)])
def test_bad_shapes_are_rejected(I, shape):
    with pytest.raises(I.IsingError) as e:
        I.batch_tuning_set(*shape)
    assert e.value.code == I.ISING_EINVAL
    assert not I.batch_tuning_get()["installed"]


def test_null_and_bad_arguments(I):
    L = I.lib()
    assert L.ising_batch_tuning_set(None) == I.ISING_EINVAL
    inst = ctypes.c_int32()
    assert L.ising_batch_tuning_get(None, ctypes.byref(inst)) == I.ISING_EINVAL
    n = ctypes.c_size_t()
    arr = (ctypes.c_void_p * 1)()
    assert L.ising_multi_autotune_bytes(arr, 0, 0, ctypes.byref(n)) == I.ISING_EINVAL
    assert L.ising_multi_autotune_bytes(arr, 0, 4, None) == I.ISING_EINVAL
    out = I.ising_batch_tuning()
    assert L.ising_multi_autotune(arr, 0, 4, None, 0, ctypes.byref(out)) == I.ISING_EINVAL
    assert L.ising_multi_autotune(arr, 1, 0, None, 0, ctypes.byref(out)) == I.ISING_EINVAL
