"""Row-strip shares (one GPU's part of the multi-GPU decomposition of
section 6), run together on one GPU with the in-process halo exchange:
they must reproduce the whole lattice's spins and per-sweep (E, M) bit for
bit, for even and uneven splits, one strip (its own halos), and at the real
share shape of 262144^2 over 8 GPUs (eight strips of 32768 rows, compared
on the device with the plain 262144^2 run, with the oracle's whole-lattice
(E, M) of tests/golden/huge_em.txt, and in light-cone windows that straddle
strip borders and the periodic wrap with the oracle)."""
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


@pytest.mark.parametrize("L,rows", [(128, [128]), (128, [64, 64]), (256, [1, 100, 155]),
                                    (1024, [300, 300, 424]), (2048, [512] * 4),
                                    (1280, [1, 1, 1278])])
def test_strips_reproduce_the_lattice(I, L, rows):
    n, beta, seed, sid = 6, 1 / 2.269185, 21, 3
    _say("case L=%d rows=%r" % (L, rows))
    st = I.StripSet(L, len(rows), seed=seed, stream_id=sid, init=workloads.INIT_HOT, beta=beta,
                    rows=rows)
    em = st.sweep_em(n).cpu().numpy()
    lat = I.Lattice(L, seed=seed, stream_id=sid, init=workloads.INIT_HOT, beta=beta)
    ref = lat.sweep_em(n).cpu().numpy()
    assert np.array_equal(em, ref)
    assert np.array_equal(st.get_spins(), lat.get_spins())
    if L <= 256:
        s, oem = oracle.run(L, beta, seed, sid, workloads.INIT_HOT, n)
        assert np.array_equal(em, oem) and np.array_equal(st.get_spins(), s)


@pytest.mark.parametrize("init,beta", [(workloads.INIT_COLD_UP, 1 / 1.5),
                                       (workloads.INIT_COLD_DOWN, 0.0)])
def test_starts_and_temperatures(I, init, beta):
    L, rows, n = 512, [128, 256, 128], 4
    st = I.StripSet(L, 3, seed=5, init=init, beta=beta, rows=rows)
    em = st.sweep_em(n).cpu().numpy()
    s, oem = oracle.run(L, beta, 5, 0, init, n)
    assert np.array_equal(em, oem) and np.array_equal(st.get_spins(), s)


def _strip_window(torch, st, L, x0, y0, ww, hh):
    """Spins (+1 / -1) of the ww x hh window at (x0, y0), periodic, read from
    the strips' packed planes: colour (x + y) & 1, own row y - y_start + 1
    (row 0 is the halo above), bit k & 63 of word k >> 6 for k = x >> 1."""
    W = L // 128
    starts = np.cumsum([0] + list(st.rows))
    out = np.empty((hh, ww), dtype=np.int8)
    for i in range(hh):
        y = (y0 + i) % L
        s = int(np.searchsorted(starts, y, side="right")) - 1
        r = st.rows[s]
        part = st.bufs[s][: 2 * (r + 2) * W * 8].view(torch.int64).view(2, r + 2, W)
        words = part[:, y - int(starts[s]) + 1].cpu().numpy().view(np.uint64)
        for j in range(ww):
            x = (x0 + j) % L
            k = x >> 1
            bit = (int(words[(x + y) & 1, k >> 6]) >> (k & 63)) & 1
            out[i, j] = 1 if bit else -1
    return out


def _golden_em(L, T, seed, sid, init):
    """{sweep: (E, M)} of the oracle's whole-lattice values for this lattice."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "huge_em.txt")
    out = {}
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if (int(f[0]), float(f[1]), int(f[2]), int(f[3]), int(f[4])) == (L, T, seed, sid, init):
            out[int(f[5])] = (int(f[6]), int(f[7]))
    return out


def test_real_share_shape(I):
    """262144^2 split over 8 GPUs: eight 32768-row strips (1 GiB each)."""
    import torch
    if torch.cuda.get_device_properties(0).total_memory < 40 * (1 << 30):
        pytest.skip("needs > 40 GiB of device memory")
    w = workloads.HUGE_T2
    L, G, n = w.L, 8, 2
    _say("case L=%d strips=%d" % (L, G))
    st = I.StripSet(L, G, seed=w.seed, stream_id=w.stream_id, init=w.init, beta=1.0 / w.T)
    em = st.sweep_em(n).cpu().numpy()
    lat = I.Lattice(L, seed=w.seed, stream_id=w.stream_id, init=w.init, beta=1.0 / w.T)
    ref = lat.sweep_em(n).cpu().numpy()
    assert np.array_equal(em, ref)
    # and the oracle's whole-lattice values (band sums, tests/golden/huge_em.txt)
    gold = _golden_em(L, w.T, w.seed, w.stream_id, w.init)
    assert len(gold) >= n
    for k in range(n):
        assert (int(em[k, 0]), int(em[k, 1])) == gold[k + 1], k
    # windows across the borders of strips 0/1 and 4/5 and across the wrap 7/0
    R = L // G
    for (x0, y0) in [(1000, R - 6), (123456, 5 * R - 3), (L - 20, L - 6)]:
        got = _strip_window(torch, st, L, x0, y0, 40, 12)
        want = oracle.window(L, 1.0 / w.T, w.seed, w.stream_id, w.init, 0, n, x0, y0, 40, 12)
        assert np.array_equal(got, want), "window at (%d, %d) differs" % (x0, y0)
    W = L // 128
    full = lat.buf[: 2 * L * W * 8].view(torch.int64).view(2, L, W)
    y0 = 0
    for buf, r in zip(st.bufs, st.rows):
        part = buf[: 2 * (r + 2) * W * 8].view(torch.int64).view(2, r + 2, W)
        assert torch.equal(part[:, 1:r + 1], full[:, y0:y0 + r]), y0
        y0 += r
    del st, lat, full
    torch.cuda.empty_cache()


def test_argument_checks(I):
    import ctypes
    assert I.lib().ising_strip_bytes(100, 10) == 0      # L % 128 != 0
    assert I.lib().ising_strip_bytes(128, 0) == 0
    assert I.lib().ising_strip_bytes(128, 129) == 0
    assert I.lib().ising_strip_bytes(128, 128) == 2 * 130 * 1 * 8 + 2 * 2048 * 8
    with pytest.raises(I.IsingError):
        I.StripSet(120, 2)
    a = I.StripSet(256, 2, rows=[100, 156], beta=0.4)
    b = I.StripSet(256, 1, beta=0.4)
    arr = (ctypes.c_void_p * 2)(a.hs[0].value, b.hs[0].value)  # rows do not tile the lattice
    with pytest.raises(I.IsingError):
        I.check(I.lib().ising_strip_exchange(arr, 2, 0))
    with pytest.raises(I.IsingError):
        I.check(I.lib().ising_strip_step(a.hs[0], 2, 0, None))
