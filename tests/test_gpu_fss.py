"""FSS analysis on the device: the reweighting kernel against the oracle on
seeded synthetic series and on oracle Metropolis series, argument checks,
and the whole chain on a batched GPU run of small lattices (the Binder
crossing lies near T_C).

Tolerance of the reweighted sums (fp64): both sides form each term with the
same operations, up to exp (within one ulp on each side), and sum them in
different orders; every sum of `count` terms is then within
(count + 8) * 2^-52 * sum|terms| of the other side's.  The shift (max x) is
computed with identical operations and compares exactly.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import fss
import physics
import workloads

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52


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


def _series(rng, L, n):
    N = L * L
    E = -4 * rng.integers(N // 8, N // 2, size=n)
    M = 2 * rng.integers(-N // 2, N // 2 + 1, size=n)
    return np.stack([E, M], axis=1).astype(np.int64)


def _check_sums(got, want, E_kept):
    cnt = len(E_kept)
    tol = (cnt + 8) * EPS
    for i in range(4):  # positive terms
        assert np.all(np.abs(got[:, i] - want[:, i]) <= tol * np.abs(want[:, i])), i
    emax = float(np.abs(E_kept).max())
    assert np.all(np.abs(got[:, 4] - want[:, 4]) <= tol * want[:, 0] * emax)


def test_reweight_matches_oracle_on_seeded_series(I):
    import torch
    rng = np.random.default_rng(21)
    specs = [(64, 57, 0, 0.44), (128, 1000, 5, 0.40), (32, 4003, 1000, 0.0), (256, 777, 700, 0.5)]
    host = [_series(rng, L, n) for (L, n, _, _) in specs]
    EMs = [torch.tensor(h, device="cuda") for h in host]
    betas0 = [b for (_, _, _, b) in specs]
    discards = [d for (_, _, d, _) in specs]
    tl, tb = [], []
    for i, b0 in enumerate(betas0):
        for db in (0.0, 0.004, -0.004, 0.02):
            tl.append(i)
            tb.append(max(b0 + db, 0.0))
    for nb in (1, 7, 20, 57):
        _say("case nblocks=%d" % nb)
        sums, shift = I.reweight(EMs, betas0, discards, tl, tb, nb)
        sums = sums.cpu().numpy()
        shift = shift.cpu().numpy()
        for k, (i, b) in enumerate(zip(tl, tb)):
            want, wshift = fss.reweight_sums(host[i][:, 0], host[i][:, 1], discards[i],
                                             betas0[i], b, nb)
            assert shift[k] == wshift, (k, shift[k], wshift)
            _check_sums(sums[k], want, host[i][discards[i]:, 0])


def test_reweight_on_two_streams(I):
    """Two reweights in flight at once on two streams, each with its own
    caller-owned work buffer; both match the oracle."""
    import torch
    rng = np.random.default_rng(77)
    host = [_series(rng, 64, 3001), _series(rng, 128, 2500)]
    EMs = [torch.tensor(h, device="cuda") for h in host]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    jobs = [(s1, 0, [0.41, 0.45, 0.43]), (s2, 1, [0.39, 0.40])]
    out = []
    for st, i, betas in jobs:
        _say("case stream %d" % i)
        tl = [0] * len(betas)
        out.append(I.reweight([EMs[i]], [0.42], [300], tl, betas, 9, stream=st))
    torch.cuda.synchronize()
    for (st, i, betas), (sums, shift) in zip(jobs, out):
        sums = sums.cpu().numpy()
        shift = shift.cpu().numpy()
        for k, b in enumerate(betas):
            want, wshift = fss.reweight_sums(host[i][:, 0], host[i][:, 1], 300, 0.42, b, 9)
            assert shift[k] == wshift
            _check_sums(sums[k], want, host[i][300:, 0])


def test_reweight_argument_checks(I):
    import torch
    EM = torch.zeros((10, 2), dtype=torch.int64, device="cuda")
    with pytest.raises(I.IsingError):
        I.reweight([EM], [0.4], [0], [0], [0.4], 11)  # more blocks than kept sweeps
    with pytest.raises(I.IsingError):
        I.reweight([EM], [0.4], [10], [0], [0.4], 1)  # nothing kept
    with pytest.raises(I.IsingError):
        I.reweight([EM], [0.4], [0], [1], [0.4], 2)  # no series 1
    with pytest.raises(I.IsingError):
        I.reweight([EM], [math.inf], [0], [0], [0.4], 2)
    with pytest.raises(I.IsingError):
        I.reweight([EM], [0.4], [0], [0], [math.nan], 2)
    # one kept sweep per block is allowed
    s, _ = I.reweight([EM], [0.4], [0], [0], [0.41], 10)
    assert np.allclose(s.cpu().numpy()[0, :, 0], 1.0)


def test_curves_from_oracle_series_match_the_oracle_chain(I):
    import torch
    temps = np.array([2.2, 2.3, 2.4])
    grid = np.linspace(2.2, 2.4, 9)
    n, d, B = 6000, 600, 12
    Ls, series = [], []
    for L in (8, 16):
        for i, T in enumerate(temps):
            _, EM = oracle.run(L, 1.0 / T, 40 + i, L, workloads.INIT_HOT, n)
            Ls.append(L)
            series.append(EM)
    temps_all = np.tile(temps, 2)
    curves = I.binder_curves([torch.tensor(s, device="cuda") for s in series], Ls, temps_all, d,
                             grid, B)
    for L in (8, 16):
        est, err, rep = curves[L]
        for k, Tf in enumerate(grid):
            runs = [j for j, v in enumerate(Ls) if v == L]
            j = runs[int(np.argmin(np.abs(temps_all[runs] - Tf)))]
            sums, _ = fss.reweight_sums(series[j][:, 0], series[j][:, 1], d, 1.0 / temps_all[j],
                                        1.0 / Tf, B)
            e, r, u = fss.jackknife(sums, L * L)
            assert np.allclose(est[k], e, rtol=1e-9, atol=1e-12)
            assert np.allclose(err[k], r, rtol=1e-6, atol=1e-12)
            assert np.allclose(rep[:, k], u, rtol=1e-9, atol=1e-12)
    a, b = curves[8], curves[16]
    got = I.binder_crossing(grid, a[0][:, 0], b[0][:, 0], a[2], b[2])
    want = fss.crossing_jackknife(grid, a[0][:, 0], b[0][:, 0], a[2], b[2])
    for g, w in zip(got, want):
        assert (math.isnan(g) and math.isnan(w)) or g == pytest.approx(w, rel=1e-12)


def test_batched_gpu_run_puts_the_binder_crossing_near_tc(I):
    """L = 8, 16, 32 at six temperatures around T_C, 2e5 sweeps each on the
    batched path; reweighted U4 curves cross within 0.03 (+ 4 errors) of
    T_C = 2/ln(1 + sqrt 2)."""
    import torch
    temps = np.linspace(2.15, 2.40, 6)
    grid = np.linspace(2.15, 2.40, 51)
    n, d, B = 200_000, 20_000, 20
    Ls, lats, EMs, T_all = [], [], [], []
    for L in (8, 16, 32):
        for i, T in enumerate(temps):
            lats.append(I.Lattice(L, seed=7 + i, stream_id=L, init=workloads.INIT_HOT,
                                  beta=1.0 / T))
            EMs.append(torch.empty((n, 2), dtype=torch.int64, device="cuda"))
            Ls.append(L)
            T_all.append(T)
    _say("case batched run, %d lattices x %d sweeps" % (len(lats), n))
    I.multi_sweep(lats, n, EMs)
    curves = I.binder_curves(EMs, Ls, T_all, d, grid, B)
    for a, b in ((8, 16), (16, 32)):
        t, u, et, eu = I.binder_crossing(grid, curves[a][0][:, 0], curves[b][0][:, 0],
                                         curves[a][2], curves[b][2])
        _say("crossing %d/%d: T* = %.4f +- %.4f, U* = %.4f +- %.4f" % (a, b, t, et, u, eu))
        assert not math.isnan(t) and not math.isnan(et)
        assert abs(t - physics.TC_EXACT) < 0.03 + 4 * et
        assert 0.55 < u < 0.68
