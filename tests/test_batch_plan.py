"""Launch-form planning of the batched path (host only, no GPU)."""
import pytest

import workloads


@pytest.fixture(scope="module")
def I():
    from paper_1007_3726_amd import ising
    ising.lib()
    return ising


CASES = [
    [g.L for g in workloads.fss_grid()],
    [4096] * 32,
    [64] * 500,
    [16384],
    [8192, 8224, 1000, 520, 40],
    [32 * k for k in range(1, 257)],
]


@pytest.mark.parametrize("Ls", CASES)
def test_plan_is_feasible(I, Ls):
    form, blocks, est = I.batch_plan(Ls, 256)
    assert form in ("fused", "packed")
    assert 1 <= blocks <= 8 * 256
    assert est > 0
    if form == "packed":
        assert blocks <= len(Ls)


def test_grid_of_large_lattices_is_fused(I):
    # the 224-lattice finite-size-scaling grid is dominated by L = 4096
    assert I.batch_plan([g.L for g in workloads.fss_grid()], 256)[0] == "fused"
    assert I.batch_plan([16384], 256)[0] == "fused"


def test_many_tiny_lattices_are_packed(I):
    assert I.batch_plan([64] * 32, 256)[0] == "packed"


def test_plan_rejects_bad_input(I):
    with pytest.raises(I.IsingError):
        I.batch_plan([6], 256)
    with pytest.raises(I.IsingError):
        I.batch_plan([64], 0)
    with pytest.raises(I.IsingError):
        I.batch_plan([], 256)
