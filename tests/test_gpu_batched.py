"""Batched sweeps (ising_multi_sweep) parity.

Every lattice advanced in the batched launches (two fused launches per
sweep over the tiles of all lattices, or one packed persistent launch for
small lattices) must be bit-identical (spins and every per-sweep (E, M)) to
the same lattice advanced alone with ising_sweep, and small members are
also checked against the CPU oracle.  Mixes cover single-workgroup packed
lattices, lattices whose tiles spread over many workgroups, partial last
words (L % 128 != 0) and lattices the tiled layout does not cover
(L % 8 != 0, plain fallback).
"""
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


def _make(I, specs):
    lats = []
    for (L, T, seed, sid, init) in specs:
        lats.append(I.Lattice(L, seed=seed, stream_id=sid, init=init, beta=1.0 / T))
    return lats


def _batched_vs_plain(I, specs, n, chunks=1, form=None, graph_chunk=-1):
    import torch
    batch = _make(I, specs)
    plain = _make(I, specs)
    EMb = [torch.empty((n, 2), dtype=torch.int64, device="cuda") for _ in specs]
    per = n // chunks
    for c in range(chunks):
        I.multi_sweep(batch, per, [e[c * per:(c + 1) * per] for e in EMb], form=form,
                      graph_chunk=graph_chunk)
    torch.cuda.synchronize()
    for i, (lat_b, lat_p) in enumerate(zip(batch, plain)):
        EMp = lat_p.sweep_em(n).cpu().numpy()
        assert np.array_equal(EMb[i].cpu().numpy(), EMp), "E/M differ for lattice %d %r" % (
            i, specs[i])
        assert np.array_equal(lat_b.get_spins(), lat_p.get_spins()), "spins differ %r" % (
            specs[i],)
        assert lat_b.sweep_count == lat_p.sweep_count == n
    return batch


MIXED = [(64, 2.2, 1, 0, 2), (128, 2.25, 1, 1, 2), (256, 2.3, 2, 2, 2), (512, 2.27, 3, 3, 2),
         (1024, 2.269, 1, 4, 2), (96, 3.0, 5, 5, 2), (160, 1.8, 6, 6, 0), (130, 2.4, 7, 7, 2),
         (6, 2.0, 8, 8, 2), (2048, 2.3, 9, 9, 2)]


@pytest.mark.parametrize("form,graph_chunk", [(None, -1), ("fused", 0), ("fused", 4),
                                              ("packed", -1)])
def test_mixed_sizes_match_plain(I, form, graph_chunk):
    _say("case mixed sizes form=%s chunk=%d" % (form, graph_chunk))
    _batched_vs_plain(I, MIXED, 24, chunks=2, form=form, graph_chunk=graph_chunk)


@pytest.mark.parametrize("specs", [
    [(4096, 2.269185, 11, 3, workloads.INIT_HOT)],  # alone: the plain path
    [(4096, 2.269185, 11, 3, workloads.INIT_HOT), (6, 2.0, 1, 1, 2)],  # with an untiled one
    [(4096, 2.2, 11, 3, workloads.INIT_HOT), (4096, 2.3, 12, 4, workloads.INIT_HOT),
     (64, 2.5, 1, 5, 2)],  # coarse fused tiles beside fine ones
])
def test_cost_model_routes_large_lattices(I, specs):
    _say("case routing %r" % ([s[0] for s in specs],))
    _batched_vs_plain(I, specs, 10, chunks=2)


@pytest.mark.parametrize("form", ["fused", "packed"])
def test_single_large_lattice(I, form):
    specs = [(4096, 2.269185, 11, 3, workloads.INIT_HOT)]
    _say("case single 4096 form=%s" % form)
    _batched_vs_plain(I, specs, 12 if form == "fused" else 3, form=form)


@pytest.mark.parametrize("form", ["fused", "packed"])
def test_wide_rows_and_partial_words(I, form):
    H = workloads.INIT_HOT
    specs = [(8192, 2.1, 1, 1, H), (8224, 2.5, 2, 2, H), (1000, 2.269, 3, 3, H),
             (520, 2.3, 4, 4, H), (40, 2.0, 5, 5, H)]
    _say("case wide and partial form=%s" % form)
    _batched_vs_plain(I, specs, 6 if form == "fused" else 2, form=form)


def test_small_members_match_oracle(I):
    import torch
    H = workloads.INIT_HOT
    specs = [(64, 2.269, 1, 0, H), (128, 2.5, 4, 2, H), (72, 1.9, 9, 1, workloads.INIT_COLD_DOWN)]
    lats = _make(I, specs)
    n = 30
    EMs = [torch.empty((n, 2), dtype=torch.int64, device="cuda") for _ in specs]
    I.multi_sweep(lats, n, EMs)
    for (L, T, seed, sid, init), lat, em in zip(specs, lats, EMs):
        s, oEM = oracle.run(L, 1.0 / T, seed, sid, init, n)
        assert np.array_equal(em.cpu().numpy(), oEM)
        assert np.array_equal(lat.get_spins(), s)


def test_fss_grid_subset_matches_plain(I):
    grid = workloads.fss_grid(sizes=[64, 128, 256, 512], temps=workloads.FSS_TEMPS[::8])
    specs = [(g.L, g.T, g.seed, g.stream_id, g.init) for g in grid]
    _say("case fss subset", len(specs))
    _batched_vs_plain(I, specs, 70, form="fused", graph_chunk=8)


def test_batched_errors(I):
    a = I.Lattice(64, beta=0.4)
    b = I.Lattice(64)
    with pytest.raises(I.IsingError):
        I.multi_sweep([a, b], 1)  # b has no beta
    with pytest.raises(I.IsingError):
        I.multi_sweep([a, a], 1)  # repeated handle
    I.multi_sweep([], 3)
    I.multi_sweep([a], 0)
    assert a.sweep_count == 0


@pytest.mark.parametrize("form", ["fused", "packed"])
def test_batched_rows_of_62_to_64_words(I, form):
    H = workloads.INIT_HOT
    specs = [(7936, 2.3, 1, 1, H), (8000, 2.4, 2, 2, H), (8064, 2.5, 3, 3, H), (96, 2.0, 4, 4, H)]
    _say("case batched W=62..63 form=%s" % form)
    _batched_vs_plain(I, specs, 2, form=form)


def _huge_golden(key):
    """{sweep: (E, M)} of tests/golden/huge_em.txt for (L, T, seed, sid, init)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "huge_em.txt")
    out = {}
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if (int(f[0]), float(f[1]), int(f[2]), int(f[3]), int(f[4])) == key:
            out[int(f[5])] = (int(f[6]), int(f[7]))
    return out


def test_lattice_totals_past_2_to_the_32(I):
    """L = 65536 from a cold start: N = 2^32 up spins, so the per-lattice
    up-spin and bond totals of the fused finaliser need 64 bits.  Batched
    per-sweep E/M equal the plain path's (64-bit per-block partials) and the
    oracle's whole-lattice values (tests/golden/huge_em.txt); spins are
    compared with the plain path and the oracle in light-cone windows (the
    full lattice is 4 GiB as int8)."""
    import torch
    L, n = 65536, 2
    spec = [(L, 2.0, 3, 1, workloads.INIT_COLD_UP)]
    _say("case L=%d fused" % L)
    b = _make(I, spec)[0]
    EMb = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    I.multi_sweep([b], n, [EMb], form="fused")
    EMb = EMb.cpu().numpy()
    p = _make(I, spec)[0]
    EMp = p.sweep_em(n).cpu().numpy()
    assert np.array_equal(EMb, EMp)
    gold = _huge_golden((L, 2.0, 3, 1, workloads.INIT_COLD_UP))
    assert sorted(gold) == [1, 2]
    for k in range(n):
        assert (int(EMb[k, 0]), int(EMb[k, 1])) == gold[k + 1], k
    assert EMp[-1, 1] > (1 << 31)  # most spins still up: the total exceeds 2^32 / 2
    for (x0, y0) in [(0, 0), (L - 40, L - 7), (L // 2, 12345)]:
        got = b.get_window(x0, y0, 64, 16)
        assert np.array_equal(got, p.get_window(x0, y0, 64, 16))
        want = oracle.window(L, 0.5, 3, 1, workloads.INIT_COLD_UP, 0, n, x0, y0, 64, 16)
        assert np.array_equal(got, want), (x0, y0)


def _grid_golden():
    """{(L, stream_id): int64 (40, 2)} oracle E/M of the grid's L >= 512 lattices."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fss_grid_em.txt")
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = [int(v) for v in line.split()]
        out[(f[0], f[1])] = np.array(f[2:], dtype=np.int64).reshape(-1, 2)
    return out


def test_whole_fss_grid_against_the_oracle(I):
    """The benchmark's 224-lattice grid (L = 64 .. 4096, 32 temperatures),
    one multi_sweep call as the benchmark makes it.  Lattices with L <= 256
    match a full oracle run (spins and per-sweep E/M); for larger ones the
    per-sweep E/M equals the oracle's whole-lattice values
    (tests/golden/fss_grid_em.txt, written from the oracle alone), the spins
    match the oracle in light-cone windows at the periodic corner and
    inside, and the last E/M equals a recount."""
    import torch
    grid = workloads.fss_grid()
    assert len(grid) == 224
    n = 40
    golden = _grid_golden()
    assert len(golden) == sum(1 for g in grid if g.L >= 512)
    _say("case whole fss grid, %d sweeps" % n)
    lats = [I.Lattice(g.L, seed=g.seed, stream_id=g.stream_id, init=g.init, beta=1.0 / g.T)
            for g in grid]
    EMs = [torch.empty((n, 2), dtype=torch.int64, device="cuda") for _ in grid]
    I.multi_sweep(lats, n, EMs)
    torch.cuda.synchronize()
    for g, lat, em in zip(grid, lats, EMs):
        em = em.cpu().numpy()
        beta = 1.0 / g.T
        if g.L <= 256:
            s, oEM = oracle.run(g.L, beta, g.seed, g.stream_id, g.init, n)
            assert np.array_equal(em, oEM), g
            assert np.array_equal(lat.get_spins(), s), g
            continue
        assert np.array_equal(em, golden[(g.L, g.stream_id)]), g
        assert lat.measure() == (int(em[-1, 0]), int(em[-1, 1])), g
        for (x0, y0) in [(g.L - 20, g.L - 6), (g.L // 3, g.L // 2 + 1)]:
            got = lat.get_window(x0, y0, 40, 12)
            want = oracle.window(g.L, beta, g.seed, g.stream_id, g.init, 0, n, x0, y0, 40, 12)
            assert np.array_equal(got, want), (g, x0, y0)


@pytest.mark.parametrize("shape", [(1, 8, 32), (4, 8, 32), (2, 4, 8), (4, 6, 64), (1, 6, 0)])
def test_every_fused_shape_matches_plain(I, shape):
    """The batched autotuner's candidate shapes (row groups per wave up to
    rpw_max, workgroups per CU, graph chunk) installed one at a time: the
    fused form stays bit-identical to the plain path.  4096^2 and 8192^2
    take four row groups per wave under rpw_max 4."""
    rpw_max, wg, chunk = shape
    H = workloads.INIT_HOT
    specs = MIXED + [(4096, 2.27, 10, 10, H), (8192, 2.4, 11, 11, H), (520, 2.3, 12, 12, H)]
    _say("case fused shape rpw_max=%d wg=%d chunk=%d" % shape)
    I.batch_tuning_set(rpw_max, wg, chunk)
    try:
        assert I.batch_tuning_get()["installed"]
        _batched_vs_plain(I, specs, 2 * chunk + 3 if chunk else 6, chunks=1, form="fused")
    finally:
        I.batch_tuning_clear()


def test_multi_autotune_installs_a_shape_and_leaves_the_lattices(I):
    import torch
    H = workloads.INIT_HOT
    specs = [(512, 2.27, 1, 1, H), (1024, 2.3, 2, 2, H), (2048, 2.25, 3, 3, H),
             (4096, 2.269, 4, 4, H), (130, 2.4, 5, 5, H), (6, 2.0, 6, 6, H)]
    lats = _make(I, specs)
    EM = [torch.empty((3, 2), dtype=torch.int64, device="cuda") for _ in specs]
    I.multi_sweep(lats, 3, EM)
    before = [(lat.get_spins(), lat.sweep_count) for lat in lats]
    _say("case multi_autotune")
    try:
        pick = I.multi_autotune(lats, 16)
        _say("pick", pick)
        for (s, c), lat in zip(before, lats):
            assert lat.sweep_count == c
            assert np.array_equal(lat.get_spins(), s)
        inst = I.batch_tuning_get()
        assert inst["installed"]
        for k in ("rpw_max", "wg_per_cu", "graph_chunk", "updates_per_ns"):
            assert inst[k] == pick[k]
        assert pick["rpw_max"] in (1, 2, 4) and 1 <= pick["wg_per_cu"] <= 8
        assert pick["updates_per_ns"] >= pick["default_updates_per_ns"] > 0
        # the installed shape gives the plain path's results
        _batched_vs_plain(I, specs, 40, chunks=2)
    finally:
        I.batch_tuning_clear()
