"""The allocation-free batched entry point (ising_multi_sweep_static),
called through the C ABI, against ising_multi_sweep with a caller work
buffer: spins and every per-sweep (E, M) bit for bit, on two calls in a row,
the second with a smaller batch; a batch whose tables exceed the static
scratch is rejected before any device work."""
import ctypes
import sys

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
    return ising


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _lattices(I, specs):
    return [I.Lattice(L, seed=seed, stream_id=sid, init=workloads.INIT_HOT, beta=1.0 / T)
            for (L, T, seed, sid) in specs]


def _arrays(lats, EMs):
    hs = (ctypes.c_void_p * len(lats))(*[lat.h.value for lat in lats])
    ems = (ctypes.c_void_p * len(lats))(*[e.data_ptr() for e in EMs])
    return hs, ems


def _check_static_against_work_buffer(I, specs, n):
    import torch
    ref = _lattices(I, specs)
    got = _lattices(I, specs)
    ref_EM = [torch.full((n, 2), -7, dtype=torch.int64, device="cuda") for _ in specs]
    got_EM = [torch.full((n, 2), -7, dtype=torch.int64, device="cuda") for _ in specs]
    hs, ems = _arrays(ref, ref_EM)
    nb = ctypes.c_size_t()
    I.check(I.lib().ising_multi_sweep_work_bytes(hs, len(specs), ctypes.byref(nb)))
    work = torch.empty(max(nb.value, 1), dtype=torch.uint8, device="cuda")
    I.check(I.lib().ising_multi_sweep(hs, len(specs), n, ems, work.data_ptr(), nb.value))
    hs2, ems2 = _arrays(got, got_EM)
    I.check(I.lib().ising_multi_sweep_static(hs2, len(specs), n, ems2))
    for spec, a, b, ea, eb in zip(specs, ref, got, ref_EM, got_EM):
        assert torch.equal(ea, eb), spec
        assert np.array_equal(a.get_spins(), b.get_spins()), spec
        assert a.sweep_count == b.sweep_count == n


def test_two_calls_second_smaller(I):
    first = [(64, 2.269, 1, 0), (256, 2.3, 2, 1), (1024, 2.2, 3, 2), (2048, 2.4, 4, 3),
             (4096, 2.269185, 5, 4), (520, 2.1, 6, 5), (40, 2.5, 7, 6)]
    second = [(128, 2.0, 8, 7), (1000, 3.0, 9, 8)]
    _say("case first call: %d lattices" % len(first))
    _check_static_against_work_buffer(I, first, 70)   # fused form, graph-sized run
    _say("case second call, smaller: %d lattices" % len(second))
    _check_static_against_work_buffer(I, second, 9)


def test_small_lattices_packed_form(I):
    specs = [(16, 2.269, 1, 0), (32, 2.3, 2, 1), (64, 2.5, 3, 2), (8, 1.5, 4, 3)]
    _say("case packed small lattices")
    _check_static_against_work_buffer(I, specs, 25)


def test_too_large_for_the_static_scratch(I):
    """16 lattices of 16384^2 need about 4.7 MB of tables (> 4 MiB)."""
    import torch
    specs = [(16384, 2.269185, i, i) for i in range(16)]
    _say("case oversized batch")
    lats = _lattices(I, specs)
    hs = (ctypes.c_void_p * len(lats))(*[lat.h.value for lat in lats])
    nb = ctypes.c_size_t()
    I.check(I.lib().ising_multi_sweep_work_bytes(hs, len(lats), ctypes.byref(nb)))
    assert nb.value > 4 << 20
    before = [lat.sweep_count for lat in lats]
    assert I.lib().ising_multi_sweep_static(hs, len(lats), 3, None) == I.ISING_ENOMEM
    assert [lat.sweep_count for lat in lats] == before
    del lats
    torch.cuda.empty_cache()
