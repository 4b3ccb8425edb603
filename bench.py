"""Benchmark of the checkerboard Metropolis sweep on one MI355X.

One step = one pass of the hot path over the HBM-resident 262144 x 262144
lattice (6.9e10 spins, 8 GiB packed 64 spins per word) at T = 2.0 from a hot
start (seed 7): 100 full sweeps with exact per-sweep int64 (E, M).  The
timed region covers exactly `--steps` steps between two synchronisations;
value is spin updates per ns (N * sweeps / time).

Also reported on the same JSON line:
  roofline      - the colour-step kernel against the integer VALU issue peak
                  (its average duration measured with HIP events on the
                  lattice's stream over the timed region);
  cpu_baseline  - the CPU oracle timed on a bounded sample of the same
                  workload (a band of rows of the same lattice, with its
                  light-cone margins) on this host's cores;
  configs       - the other plain configurations: the same lattice at
                  T = 3.0, 16384^2 at T = 2.269185 from a cold start (2000
                  sweeps, in the 256 MB Infinity Cache), and 64^2 at T = 2.269
                  (1000 sweeps, its latency);
  lcg, pool     - the 16384^2 workload with the paper's own random numbers:
                  per-thread LCGs, and Boltzmann-pattern pools read at random
                  addresses or linearly;
  strip_share   - one GPU's share of 262144^2 split over 8 GPUs (a 32768-row
                  strip with halo rows), all eight strips run here;
  table2        - the paper's benchmark point (4096^2 at 0.99 T_C) with every
                  update variant, batched, and the multi-spin CPU baseline;
  batched       - the 224-lattice finite-size-scaling grid advanced together,
                  with its Binder-cumulant analysis (crossings only where the
                  series are long against their autocorrelation times);
  fss_proof     - long runs of small lattices whose crossing locates T_C;
  served        - the 2000-request Poisson stream with continuous batching
                  (aggregate rate, p50/p99 latency) and its first requests
                  one at a time on the plain path;
  cpu_msc       - the multi-spin-coded CPU baseline (same chain, 64 spins per
                  word, vectorised Philox) on the 16384^2 lattice.

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 1]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations/s.
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# Algorithmic lane-operations per spin update:
# a quarter of a Philox4x32-10 block (10 rounds x (2 wide multiplies + 2
# three-input XORs) / 4 = 10), two threshold compares and two bit inserts.
ALU_OPS_PER_UPDATE = 14.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-rows", type=int, default=16384,
                   help="rows of the lattice in the CPU oracle's sample (a band with light-cone "
                        "margins, 2 sweeps) for the 262144^2 workloads")
    p.add_argument("--cpu-sweeps", type=int, default=16,
                   help="sweeps the oracle runs for the CPU baseline of the smaller workloads")
    p.add_argument("--sweeps", type=int, default=None,
                   help="sweeps per step (default: the workload's 2000); for short profiles")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a plain 1 GiB device copy, the reference for HBM counters")
    p.add_argument("--no-batched", action="store_true",
                   help="skip the batched finite-size-scaling grid")
    p.add_argument("--batched-sweeps", type=int, default=workloads.FSS_SWEEPS)
    p.add_argument("--no-fss-proof", action="store_true",
                   help="skip the long small-lattice runs of the FSS proof of concept")
    p.add_argument("--workload", default="huge-T2",
                   choices=["large", "huge-T2", "huge-T3", "small", "paper-4096"],
                   help="plain workload: huge = 262144^2 (8 GiB, HBM-resident; T2 is the "
                        "headline), large = 16384^2, small = 64^2, paper-4096 = 4096^2 at "
                        "0.99 T_c")
    p.add_argument("--no-configs", action="store_true",
                   help="skip the other plain configurations")
    p.add_argument("--side-workload", default="large", choices=["large", "headline"],
                   help="lattice of the LCG, pattern-pool and multi-spin CPU legs: 16384^2 "
                        "(default) or the headline workload")
    p.add_argument("--no-served", action="store_true", help="skip the served request stream")
    p.add_argument("--no-cpu-msc", action="store_true",
                   help="skip the multi-spin-coded CPU baseline")
    p.add_argument("--no-lcg", action="store_true",
                   help="skip the plain workload with the paper's LCG random numbers")
    p.add_argument("--no-strip", action="store_true",
                   help="skip the row-strip share (one GPU's part of 262144^2 over 8 GPUs)")
    p.add_argument("--no-table2", action="store_true",
                   help="skip the paper's 4096^2 benchmark point with every variant")
    p.add_argument("--no-pool", action="store_true",
                   help="skip the plain workload with Boltzmann-pattern pools")
    p.add_argument("--no-autotune", action="store_true",
                   help="skip the autotuners (profiling runs: no trial launches)")
    p.add_argument("--batched-shape", default=None,
                   help="rpw_max,wg_per_cu,graph_chunk of the batched grid's fused launches "
                        "instead of the batched autotuner's pick (profiling runs)")
    p.add_argument("--served-requests", type=int, default=2000,
                   help="requests of the 2000-request Poisson stream to serve (default: all, "
                        "about 160 s; 0: only the capacity and plain-FIFO samples)")
    p.add_argument("--served-capacity", type=int, default=300,
                   help="requests of the stream queued at once to measure the server's capacity")
    p.add_argument("--served-arena-gib", type=float, default=1.0)
    p.add_argument("--served-quantum", type=int, default=400)
    p.add_argument("--plain-fifo-requests", type=int, default=200,
                   help="requests of the same stream run one by one with the plain path")
    return p.parse_args()


def _serve_stream(ising, dev, stream, arena_gib, quantum):
    """Serve the requests at their scheduled arrival times; aggregate rate
    and latencies."""
    srv = ising.Server(int(arena_gib * (1 << 30)), quantum_sweeps=quantum, device=dev)
    t0 = time.perf_counter()
    t0_abs = _monotonic_now()
    nxt = 0
    pending = {}
    lat = []
    work_done = 0
    t_last = 0.0
    last_note = time.perf_counter()
    while nxt < len(stream) or pending:
        now = time.perf_counter() - t0
        if time.perf_counter() - last_note > 5.0:
            print("bench: served t=%.0fs submitted=%d finished=%d in flight=%d"
                  % (now, nxt, len(lat), len(pending)), file=sys.stderr, flush=True)
            last_note = time.perf_counter()
        batch = []
        while nxt < len(stream) and stream[nxt].arrival <= now:
            batch.append(stream[nxt])
            nxt += 1
        if batch:
            reqs = [{"L": r.L, "beta": 1.0 / r.T, "seed": r.seed, "stream_id": r.stream_id,
                     "init": r.init, "n_sweeps": r.sweeps, "n_discard": r.sweeps // 5}
                    for r in batch]
            for r, t in zip(batch, srv.submit(reqs)):
                pending[t] = r
        busy = srv.step() if pending else False
        for t in list(pending):
            res = srv.poll(t)
            if res is not None:
                r = pending.pop(t)
                # latency from the scheduled arrival (queueing included)
                lat.append(res["t_done"] - (t0_abs + r.arrival))
                work_done += r.L * r.L * r.sweeps
                t_last = max(t_last, res["t_done"])
        if not busy and not pending and nxt < len(stream):
            time.sleep(max(0.0, stream[nxt].arrival - (time.perf_counter() - t0)))
    wall = t_last - (t0_abs + stream[0].arrival)
    stats = srv.stats()
    srv.close()
    lat = np.array(lat)
    return {"value": round(work_done / (wall * 1e9), 2),
            "p50_latency_s": round(float(np.percentile(lat, 50)), 3),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 3),
            "mean_latency_s": round(float(lat.mean()), 3),
            "wall_s": round(wall, 3),
            "peak_arena_bytes": stats["peak_bytes"], "quanta": stats["quanta"],
            "valu_roof_frac": round(work_done / (wall * 1e9) * ALU_OPS_PER_UPDATE * 1e9
                                    / VALU_PEAK_LANE_OPS, 4)}


def bench_served(torch, ising, dev, n_req, arena_gib, quantum, plain_n, plain_rate, cap_n=300):
    """Poisson stream of requests (L log-uniform in [32, 8192], T uniform in
    [1.5, 3.5], sweeps log-uniform in [1e3, 1e5], seed 1000 + i, hot start)
    served with continuous batching; arrival rate 0.7 x the plain throughput
    divided by the mean work per request (1.30e11 spin updates).  Also the
    server's capacity on the stream's first cap_n requests queued at once,
    and the first plain_n requests run one at a time on the plain path."""
    import numpy as np
    rate = 0.7 * plain_rate * 1e9 / 1.30e11
    full = workloads.served_stream(2000, rate=rate)
    stream = full[:n_req]
    out = {"unit": "spin updates/ns", "requests": len(stream), "rate_per_s": round(rate, 3),
           "arena_gib": arena_gib, "quantum_sweeps": quantum}
    if stream:
        out.update(_serve_stream(ising, dev, stream, arena_gib, quantum))
    # capacity: the first requests of the stream all queued at once, so the
    # server never waits for an arrival
    if cap_n > 0:
        print("bench: served capacity (%d requests queued at once)" % cap_n, file=sys.stderr,
              flush=True)
        sub = full[:cap_n]
        srv = ising.Server(int(arena_gib * (1 << 30)), quantum_sweeps=quantum, device=dev)
        reqs = [{"L": r.L, "beta": 1.0 / r.T, "seed": r.seed, "stream_id": r.stream_id,
                 "init": r.init, "n_sweeps": r.sweeps, "n_discard": r.sweeps // 5} for r in sub]
        torch.cuda.synchronize()
        tc = time.perf_counter()
        tickets = srv.submit(reqs)
        srv.run_until_idle()
        dtc = time.perf_counter() - tc
        done = [srv.poll(t) for t in tickets]
        assert all(d is not None for d in done)
        srv.close()
        cwork = sum(r.L * r.L * r.sweeps for r in sub)
        out["capacity"] = {"requests": cap_n, "value": round(cwork / (dtc * 1e9), 2),
                           "seconds": round(dtc, 3),
                           "valu_roof_frac": round(cwork / dtc * ALU_OPS_PER_UPDATE
                                                   / VALU_PEAK_LANE_OPS, 4)}
    # the same requests one at a time through the plain path (FIFO, no overlap)
    if plain_n > 0:
        sub = full[:plain_n]
        tp = time.perf_counter()
        clock = 0.0
        plat = []
        pwork = 0
        for j, r in enumerate(sub):
            if j % 5 == 0:
                print("bench: plain FIFO request %d/%d" % (j, plain_n), file=sys.stderr,
                      flush=True)
            L = ising.Lattice(r.L, seed=r.seed, stream_id=r.stream_id, init=r.init,
                              beta=1.0 / r.T, device=dev)
            torch.cuda.synchronize()
            a = time.perf_counter()
            L.sweep(r.sweeps)
            torch.cuda.synchronize()
            svc = time.perf_counter() - a
            clock = max(clock, r.arrival) + svc
            plat.append(clock - r.arrival)
            pwork += r.L * r.L * r.sweeps
            del L
        busy_s = time.perf_counter() - tp
        plat = np.array(plat)
        out["plain_fifo"] = {"requests": plain_n, "value": round(pwork / (clock - sub[0].arrival)
                                                                 / 1e9, 2),
                             "service_rate": round(pwork / (busy_s * 1e9), 2),
                             "p50_latency_s": round(float(np.percentile(plat, 50)), 3),
                             "p99_latency_s": round(float(np.percentile(plat, 99)), 3)}
    return out


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("ising_device.hpp", "ising_kernels.hpp", "ising_kernels.hip"):
        with open(os.path.join(ROOT, "paper_1007_3726_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def plain_kernel(ising, L, tuned):
    """Name of the kernel that runs a colour step of the plain sweep for side L
    under the tuning entry `tuned`."""
    if 2 * L * ((L // 2 + 63) // 64) * 8 <= tuned["small_lds_bytes"]:
        return "k_small_sweeps"
    if tuned["form"] == ising.ISING_FORM_STRIP and (L // 2 + 63) // 64 >= 63:
        return "k_strip_sweep"
    return "k_tile_sweep"


def profiled_traffic(kernel, L):
    """HBM bytes per launch from the committed rocprofv3 summary of this kernel
    and lattice side (FETCH_SIZE + WRITE_SIZE scaled by a plain copy), or None
    when the summary is missing or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "%s_plain-%d.txt" % (kernel, L))
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ": " in line and not line.startswith(("#", " ", "|")):
                k, v = line.rstrip("\n").split(": ", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_sources_sha():
        return None
    try:
        return int(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _monotonic_now():
    """The library's clock for t_arrive/t_admit/t_done (steady clock, seconds)."""
    return time.monotonic()


def binder_exact(M, discard):
    """U4 = 1 - <M^4> / (3 <M^2>^2) from an int64 series, with exact integer sums."""
    from fractions import Fraction
    m = [int(v) for v in M[discard:]]
    n = len(m)
    s2 = sum(v * v for v in m)
    s4 = sum(v ** 4 for v in m)
    return float(1 - Fraction(s4 * n, 3 * s2 * s2)) if s2 else float("nan")


# A series supports an error estimate (the reading taken here; the paper
# gives none) when Sokal's window converged, each of the jackknife blocks
# spans at least BLOCK_TAUS integrated autocorrelation times of M^2, and the
# discarded start spans at least DISCARD_TAUS of them.
BLOCK_TAUS = 10.0
DISCARD_TAUS = 20.0


def series_check(ising, M, discard, nblocks):
    """(ok, tau, window) for the kept part of an int64 magnetisation series."""
    kept = np.asarray(M[discard:], dtype=np.float64)
    tau, W = ising.autocorr_time(kept * kept)
    per_block = len(kept) / nblocks
    ok = W > 0 and per_block >= BLOCK_TAUS * tau and discard >= DISCARD_TAUS * tau
    return bool(ok), float(tau), int(W)


def crossings_where_resolved(ising, sizes, checks, fine, curves):
    """Binder crossings of adjacent sizes, reported only where every run of
    both sizes passes series_check; otherwise the reason."""
    out = {}
    for x, y in zip(sizes[:-1], sizes[1:]):
        key = "%d/%d" % (x, y)
        bad = [(L, c) for L in (x, y) for c in checks[L] if not c[0]]
        if bad:
            worst = max(bad, key=lambda v: v[1][1])
            out[key] = {"resolved": False,
                        "reason": "%d of %d runs too short for their autocorrelation "
                                  "(largest tau_int of M^2: %.0f sweeps at L=%d)"
                                  % (len(bad), len(checks[x]) + len(checks[y]), worst[1][1],
                                     worst[0])}
            continue
        t, u, et, eu = ising.binder_crossing(fine, curves[x][0][:, 0], curves[y][0][:, 0],
                                             curves[x][2], curves[y][2])
        out[key] = {"resolved": True, "T": round(t, 5), "T_err": round(et, 5),
                    "U4": round(u, 4), "U4_err": round(eu, 4)}
    return out


def bench_batched(torch, ising, dev, sweeps, autotune=True):
    """224 lattices (L in 64..4096 x 32 temperatures) advanced together:
    two fused launches per sweep over all lattices, replayed from captured
    hipGraph chunks, in the fused shape the batched autotuner picks on
    copies of the same lattices."""
    grid = workloads.fss_grid()
    lats = [ising.Lattice(g.L, seed=g.seed, stream_id=g.stream_id, init=g.init, beta=1.0 / g.T,
                          device=dev) for g in grid]
    EMs = [torch.empty((sweeps, 2), dtype=torch.int64, device=dev) for _ in grid]
    pick = None
    if autotune:
        t_tune = time.perf_counter()
        pick = ising.multi_autotune(lats, 128)
        pick = {k: (round(v, 1) if isinstance(v, float) else v) for k, v in pick.items()}
        pick["seconds"] = round(time.perf_counter() - t_tune, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ising.multi_sweep(lats, sweeps, EMs)  # synchronises
    dt = time.perf_counter() - t0
    updates = sum(g.L * g.L for g in grid) * sweeps
    discard = min(workloads.FSS_DISCARD, sweeps // 5)
    binder = {}
    for g, em in zip(grid, EMs):
        binder.setdefault(g.L, []).append(binder_exact(em[:, 1].cpu().numpy(), discard))
    # the same lattices advanced one by one with the plain path (rate sample)
    plain_sweeps = max(1, min(sweeps, 500))
    seq = [ising.Lattice(g.L, seed=g.seed, stream_id=g.stream_id, init=g.init, beta=1.0 / g.T,
                         device=dev) for g in grid]
    plain_EMs = [torch.empty((plain_sweeps, 2), dtype=torch.int64, device=dev) for _ in grid]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for lat, em in zip(seq, plain_EMs):
        lat.sweep(plain_sweeps, em)
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t1
    plain_updates = sum(g.L * g.L for g in grid) * plain_sweeps
    for em, pem in zip(EMs, plain_EMs):
        assert torch.equal(em[:plain_sweeps], pem), "batched and plain series differ"
    del seq, plain_EMs
    tidx = [0, len(workloads.FSS_TEMPS) // 2, len(workloads.FSS_TEMPS) - 1]
    fss = bench_fss(torch, ising, dev, grid, EMs, discard)
    return {
        "value": round(updates / (dt * 1e9), 2), "unit": "spin updates/ns",
        "valu_roof_frac": round(updates / dt * ALU_OPS_PER_UPDATE / VALU_PEAK_LANE_OPS, 4),
        "workload": "224 lattices, L in {64..4096} x 32 T in [2.20, 2.34], hot start, "
                    "%d sweeps each, per-sweep int64 E/M; two fused launches per sweep over "
                    "all lattices, replayed from hipGraph chunks" % sweeps,
        "seconds": round(dt, 3),
        "shape": {k: v for k, v in ising.batch_tuning_get().items()
                  if k in ("rpw_max", "wg_per_cu", "graph_chunk", "installed")},
        "autotuner_pick": pick,
        "plain_one_by_one": {"value": round(plain_updates / (dt_plain * 1e9), 2),
                             "sweeps": plain_sweeps},
        "binder_U4": {str(L): {"%.4f" % workloads.FSS_TEMPS[i]: round(v[i], 4) for i in tidx}
                      for L, v in binder.items()},
        "discard": discard,
        "fss": fss,
    }


def bench_fss(torch, ising, dev, grid, EMs, discard, per_interval=8, nblocks=20):
    """Binder cumulants of the batched grid reweighted on the device to a
    grid 8x finer than the simulated temperatures (each point from the
    nearest run), with jackknife errors; crossings of adjacent sizes only
    where the series are long against their autocorrelation times."""
    temps = np.array([g.T for g in grid])
    Ls = [g.L for g in grid]
    T_lo, T_hi = float(temps.min()), float(temps.max())
    n_sim = len(workloads.FSS_TEMPS)
    fine = np.linspace(T_lo, T_hi, (n_sim - 1) * per_interval + 1)
    stream = torch.cuda.current_stream(dev)
    # time the reweighting kernel alone on the stream it runs on
    tl, tb = [], []
    for L in sorted(set(Ls)):
        runs = [i for i, v in enumerate(Ls) if v == L]
        for T in fine:
            tl.append(runs[int(np.argmin(np.abs(temps[runs] - T)))])
            tb.append(1.0 / T)
    ising.reweight(EMs, [1.0 / t for t in temps], [discard] * len(EMs), tl, tb, nblocks, stream)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    ising.reweight(EMs, [1.0 / t for t in temps], [discard] * len(EMs), tl, tb, nblocks, stream)
    b.record(stream)
    b.synchronize()
    rw_ms = a.elapsed_time(b)
    t0 = time.perf_counter()
    curves = ising.binder_curves(EMs, Ls, temps, discard, fine, nblocks, stream)
    checks = {}
    for L, em in zip(Ls, EMs):
        checks.setdefault(L, []).append(series_check(ising, em[:, 1].cpu().numpy(), discard,
                                                     nblocks))
    sizes = sorted(curves)
    cross = crossings_where_resolved(ising, sizes, checks, fine, curves)
    chain_s = time.perf_counter() - t0
    samples = EMs[0].shape[0] - discard
    return {"grid_points": len(fine), "tasks": len(tl), "samples_per_task": int(samples),
            "nblocks": nblocks, "reweight_ms": round(rw_ms, 3),
            "reweight_samples_per_s": round(len(tl) * samples / (rw_ms * 1e-3), 1),
            "analysis_s": round(chain_s, 3),
            "tau_int_M2_max": {str(L): round(max(c[1] for c in checks[L]), 1) for L in sizes},
            "runs_resolved": {str(L): sum(c[0] for c in checks[L]) for L in sizes},
            "crossings": cross,
            "tc_exact": round(2.0 / math.log(1.0 + math.sqrt(2.0)), 6)}


# The paper's per-thread LCG dynamics: one v_mad_u64_u32 per uniform (the
# chain runs on a shifted state so that the first range test is a bare
# compare), one add for the second range test, two compares and two bit
# inserts: 6 lane-operations per spin update.
LCG_OPS_PER_UPDATE = 6.0


def bench_lcg(torch, ising, dev, w, steps):
    """The plain workload with the paper's own random numbers (section 5.3)."""
    lat = ising.Lattice(w.L, seed=w.seed, stream_id=w.stream_id, init=w.init, beta=1.0 / w.T,
                        device=dev)
    lat.use_lcg()
    EM = torch.empty((w.sweeps, 2), dtype=torch.int64, device=dev)
    stream = lat.stream
    lat.sweep(w.sweeps, EM)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        lat.sweep(w.sweeps, EM)
    b.record(stream)
    b.synchronize()
    ms = a.elapsed_time(b)
    N = w.L * w.L
    launch_us = ms * 1e3 / (2 * w.sweeps * steps)
    achieved = LCG_OPS_PER_UPDATE * (N / 2) / (launch_us * 1e-6)
    last = EM[-1].cpu().tolist()
    assert tuple(last) == lat.measure(), "fused E/M disagrees with a recount"
    return {"value": round(N * w.sweeps * steps / (ms * 1e6), 2), "unit": "spin updates/ns",
            "workload": "as the plain workload, per-thread LCG x <- 1664525 x + 1013904223 "
                        "mod 2^32 per 64-site word (Eqs. (6), (7))",
            "avg_launch_us": round(launch_us, 3), "ops_per_update": LCG_OPS_PER_UPDATE,
            "roofline_frac": round(achieved / VALU_PEAK_LANE_OPS, 4)}


# Algorithmic HBM bytes per update of the pattern-pool dynamics: the two
# colour planes (3 bits: read both colours once, write one) plus one
# 16-byte (r4, r8) pattern pair per 64-site word.
POOL_BYTES_PER_UPDATE = 3 / 8 + 16 / 64
HBM_PEAK_BYTES = 8.0e12


def bench_pool(torch, ising, dev, w, steps, log2_patterns=22):
    """The plain workload with section 4's Boltzmann-pattern pool instead of
    per-site uniforms: a random pool address per word (Table 2's
    "unmodified" GPU variant) and linear reads from one random start per
    256 words (its "linear" variant)."""
    out = {"log2_patterns": log2_patterns,
           "pool_bytes": ising.ising_pool_bytes(log2_patterns),
           "bytes_per_update": POOL_BYTES_PER_UPDATE}
    N = w.L * w.L
    for name, linear in (("random", False), ("linear", True)):
        lat = ising.Lattice(w.L, seed=w.seed, stream_id=w.stream_id, init=w.init,
                            beta=1.0 / w.T, device=dev)
        lat.use_pool(log2_patterns, linear)
        EM = torch.empty((w.sweeps, 2), dtype=torch.int64, device=dev)
        stream = lat.stream
        lat.sweep(w.sweeps, EM)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            lat.sweep(w.sweeps, EM)
        b.record(stream)
        b.synchronize()
        ms = a.elapsed_time(b)
        assert tuple(EM[-1].cpu().tolist()) == lat.measure(), "E/M disagrees with a recount"
        ups = N * w.sweeps * steps / (ms * 1e6)
        out[name] = {"value": round(ups, 2), "unit": "spin updates/ns",
                     "avg_launch_us": round(ms * 1e3 / (2 * w.sweeps * steps), 3),
                     "hbm_frac": round(ups * 1e9 * POOL_BYTES_PER_UPDATE / HBM_PEAK_BYTES, 4)}
        del lat, EM
        torch.cuda.empty_cache()
    return out


def bench_table2(torch, ising, dev, reps=3):
    """The paper's benchmark point (Table 2: one 4096^2 lattice at
    T = 0.99 T_C) with every update variant built here, and 32 such lattices
    batched, against the multi-spin-coded CPU baseline on this host."""
    w = workloads.PAPER_POINT
    N = w.L * w.L

    def gpu_rate(setup):
        lat = ising.Lattice(w.L, seed=w.seed, stream_id=w.stream_id, init=w.init,
                            beta=1.0 / w.T, device=dev)
        setup(lat)
        EM = torch.empty((w.sweeps, 2), dtype=torch.int64, device=dev)
        lat.sweep(w.sweeps, EM)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(lat.stream)
        for _ in range(reps):
            lat.sweep(w.sweeps, EM)
        b.record(lat.stream)
        b.synchronize()
        return round(N * w.sweeps * reps / (a.elapsed_time(b) * 1e6), 2)

    rows = {"gpu_philox_on_the_fly": gpu_rate(lambda lat: None),
            "gpu_lcg_on_the_fly": gpu_rate(lambda lat: lat.use_lcg()),
            "gpu_pool_random_addresses": gpu_rate(lambda lat: lat.use_pool(22, False)),
            "gpu_pool_linear": gpu_rate(lambda lat: lat.use_pool(22, True))}
    lats = [ising.Lattice(w.L, seed=w.seed, stream_id=i, init=w.init, beta=1.0 / w.T,
                          device=dev) for i in range(32)]
    EMs = [torch.empty((w.sweeps, 2), dtype=torch.int64, device=dev) for _ in lats]
    ising.multi_sweep(lats, w.sweeps, EMs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ising.multi_sweep(lats, w.sweeps, EMs)
    torch.cuda.synchronize()
    rows["gpu_batched_32_lattices"] = round(32 * N * w.sweeps * reps /
                                            ((time.perf_counter() - t0) * 1e9), 2)
    del lats, EMs
    import baselines
    msc = baselines.Lattice(w.L, seed=w.seed, stream_id=w.stream_id, init=w.init)
    msc.sweeps(1.0 / w.T, 2, record=True)
    t0 = time.perf_counter()
    msc.sweeps(1.0 / w.T, w.sweeps, record=True)
    rows["cpu_msc_all_cores"] = round(N * w.sweeps / ((time.perf_counter() - t0) * 1e9), 3)
    one = baselines.Lattice(w.L, seed=w.seed, stream_id=w.stream_id, init=w.init, threads=1)
    t0 = time.perf_counter()
    one.sweeps(1.0 / w.T, 20, record=True)
    rows["cpu_msc_1_core"] = round(N * 20 / ((time.perf_counter() - t0) * 1e9), 3)
    # the paper's own CPU scheme: Boltzmann-pattern pool (2^22 patterns)
    for name, linear in (("random_addresses", False), ("linear", True)):
        msc.use_pool(1.0 / w.T, 22, linear)
        t0 = time.perf_counter()
        msc.pool_sweeps(w.sweeps, record=True)
        rows["cpu_msc_pool_%s_all_cores" % name] = round(
            N * w.sweeps / ((time.perf_counter() - t0) * 1e9), 3)
        one.use_pool(1.0 / w.T, 22, linear)
        t0 = time.perf_counter()
        one.pool_sweeps(10, record=True)
        rows["cpu_msc_pool_%s_1_core" % name] = round(
            N * 10 / ((time.perf_counter() - t0) * 1e9), 3)
    return {"workload": "%dx%d, T = 0.99 T_C = %.6f, hot start, %d sweeps per run with per-sweep "
                        "E/M" % (w.L, w.L, w.T, w.sweeps),
            "unit": "spin updates/ns", "rows": rows,
            "cpu_cores": int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()}


def bench_strip_share(torch, ising, dev, nstrips=8, sweeps=3):
    """One GPU's share of the row-strip decomposition at its real shape:
    262144^2 over 8 GPUs is eight strips of 32768 rows.  All eight run here
    on one GPU; reported are one strip's colour-step kernel (the per-GPU
    work), the in-process halo exchange of one colour, and the whole set's
    rate, against the plain 262144^2 sweep."""
    w = workloads.HUGE_T2
    st = ising.StripSet(w.L, nstrips, seed=w.seed, stream_id=w.stream_id, init=w.init,
                        beta=1.0 / w.T, device=dev)
    st.sweep_em(1)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    stream = st.stream
    ev[0].record(stream)
    st.sweep_em(sweeps)
    ev[1].record(stream)
    ev[1].synchronize()
    total_ms = ev[0].elapsed_time(ev[1])
    # one strip's colour-0 step, then one colour's exchange
    ev[2].record(stream)
    ising.check(ising.lib().ising_strip_step(st.hs[0], 0, st.t, None))
    ev[3].record(stream)
    ev[3].synchronize()
    step_ms = ev[2].elapsed_time(ev[3])
    ev[2].record(stream)
    ising.check(ising.lib().ising_strip_exchange(st._arr, nstrips, 0))
    ev[3].record(stream)
    ev[3].synchronize()
    exch_ms = ev[2].elapsed_time(ev[3])
    share_updates = (w.L // nstrips) * w.L // 2
    out = {"workload": "%dx%d split into %d strips of %d rows (one GPU's share each), T=%r, "
                       "hot start" % (w.L, w.L, nstrips, w.L // nstrips, w.T),
           "share_colour_step_us": round(step_ms * 1e3, 1),
           "share_updates_per_ns": round(share_updates / (step_ms * 1e6), 1),
           "exchange_us_per_colour": round(exch_ms * 1e3, 1),
           "all_strips_updates_per_ns": round(w.L * w.L * sweeps / (total_ms * 1e6), 1),
           "halo_bytes_per_strip_per_colour": 2 * (w.L // 128) * 8}
    del st
    torch.cuda.empty_cache()
    return out


def bench_fss_proof(torch, ising, dev, sweeps=200_000, discard=20_000, nblocks=20):
    """The paper's proof of concept (section 2): Binder cumulants of small
    lattices (L = 8..64, six temperatures in [2.15, 2.40], long runs on the
    batched path) cross near T_C; crossings only where the series are long
    against their autocorrelation times."""
    temps = np.linspace(2.15, 2.40, 6)
    sizes = (8, 16, 32, 64)
    lats, EMs, Ls, T_all = [], [], [], []
    for L in sizes:
        for i, T in enumerate(temps):
            lats.append(ising.Lattice(L, seed=7 + i, stream_id=L, init=workloads.INIT_HOT,
                                      beta=1.0 / T, device=dev))
            EMs.append(torch.empty((sweeps, 2), dtype=torch.int64, device=dev))
            Ls.append(L)
            T_all.append(T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ising.multi_sweep(lats, sweeps, EMs)
    dt = time.perf_counter() - t0
    fine = np.linspace(2.15, 2.40, 51)
    curves = ising.binder_curves(EMs, Ls, T_all, discard, fine, nblocks)
    checks = {}
    for L, em in zip(Ls, EMs):
        checks.setdefault(L, []).append(series_check(ising, em[:, 1].cpu().numpy(), discard,
                                                     nblocks))
    cross = crossings_where_resolved(ising, list(sizes), checks, fine, curves)
    return {"workload": "L in {8,16,32,64} x 6 T in [2.15, 2.40], hot start, %d sweeps, "
                        "discard %d" % (sweeps, discard),
            "seconds": round(dt, 3),
            "updates_per_ns": round(sum(L * L for L in Ls) * sweeps / (dt * 1e9), 2),
            "tau_int_M2_max": {str(L): round(max(c[1] for c in checks[L]), 1) for L in sizes},
            "crossings": cross,
            "tc_exact": round(2.0 / math.log(1.0 + math.sqrt(2.0)), 6)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_msc(w, gpu_value, seconds=2.0):
    """The multi-spin-coded CPU baseline on the workload's lattice: all-core
    rate over about `seconds` of sweeps, and the one-core rate of one sweep."""
    import baselines
    lat = baselines.Lattice(w.L, seed=w.seed, stream_id=w.stream_id, init=w.init)
    beta = 1.0 / w.T
    t0 = time.perf_counter()
    lat.sweeps(beta, 1, record=True)
    first = time.perf_counter() - t0
    n = max(1, min(200, int(seconds / max(first, 1e-6))))
    t0 = time.perf_counter()
    lat.sweeps(beta, n, record=True)
    dt = time.perf_counter() - t0
    ups = w.L * w.L * n / (dt * 1e9)
    one = baselines.Lattice(w.L, seed=w.seed, stream_id=w.stream_id, init=w.init, threads=1)
    t1 = time.perf_counter()
    one.sweeps(beta, 1, record=True)
    dt1 = time.perf_counter() - t1
    ups1 = w.L * w.L / (dt1 * 1e9)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": ups, "unit": "spin updates/ns", "cores": threads, "kind": "msc-cpu",
            "value_1core": ups1,
            "philox": "avx512" if baselines.vector_available() and w.L % 8 == 0 else "scalar",
            "sample": "%d sweeps of the %dx%d lattice after one untimed (%.1f s); one core: "
                      "1 sweep (%.1f s)" % (n, w.L, w.L, dt, dt1),
            "cpu_model": cpu_model(),
            "gpu_over_cpu": round(gpu_value / ups, 1)}


def cpu_baseline(w, sweeps, band_rows):
    """The CPU oracle on a bounded sample of workload w, on this host's cores.
    For lattices too large for it to hold (262144^2 would take 69 GB at one
    byte per spin) the sample is a band of rows of the same lattice simulated
    with its light-cone margins (oracle.band_em, 2 sweeps from the start);
    the rate counts the sites swept, and the time of the start alone (the
    same call with no sweeps) is taken off."""
    import oracle
    threads = oracle.get_threads()
    kind = ["cold +1", "cold -1", "hot"][w.init]
    one = None
    if w.L > 65536:
        n = 2

        def band(rows):
            t0 = time.perf_counter()
            oracle.band_em(w.L, 1.0 / w.T, w.seed, w.stream_id, w.init, 0, 0, 0, rows)
            t_start = time.perf_counter() - t0
            t0 = time.perf_counter()
            oracle.band_em(w.L, 1.0 / w.T, w.seed, w.stream_id, w.init, 0, n, 0, rows)
            dt = time.perf_counter() - t0 - t_start
            swept = (rows + 2 * (2 * n + 1) - 2) * w.L * n
            return swept, dt, t_start

        rows = min(band_rows, w.L - 2 * (2 * n + 1))
        swept, dt, t_start = band(rows)
        ups = swept / (dt * 1e9)
        sample = ("%d sweeps of rows 0..%d of the %dx%d lattice (%s start, T=%r) with their "
                  "%d-row light-cone margins: %.2e site updates in %.1f s (the start, %.1f s, "
                  "not counted)" % (n, rows - 1, w.L, w.L, kind, w.T, 2 * n + 1, swept, dt,
                                    t_start))
        # one core on a band 1/32 as tall
        oracle.set_threads(1)
        try:
            rows1 = max(rows // 32, 1)
            swept1, dt1, _ = band(rows1)
        finally:
            oracle.set_threads(threads)
        one = {"value": round(swept1 / (dt1 * 1e9), 4),
               "sample": "the same on rows 0..%d, one thread: %.2e site updates in %.1f s"
                         % (rows1 - 1, swept1, dt1)}
    else:
        s = oracle.init(w.L, w.seed, w.stream_id, w.init)
        t0 = time.perf_counter()
        oracle.sweeps(s, 1.0 / w.T, w.seed, w.stream_id, 0, sweeps, record=True)
        dt = time.perf_counter() - t0
        ups = w.L * w.L * sweeps / (dt * 1e9)
        sample = "%d sweeps of the %dx%d lattice (%s start, T=%r), %.1f s" % (
            sweeps, w.L, w.L, kind, w.T, dt)
    # the paper's benchmark point (Table 2's "CPU simple" row: one byte per
    # spin), all cores and one core
    p = workloads.PAPER_POINT
    sp = oracle.init(p.L, p.seed, p.stream_id, p.init)
    t1 = time.perf_counter()
    oracle.sweeps(sp, 1.0 / p.T, p.seed, p.stream_id, 0, 10, record=True)
    paper_all = p.L * p.L * 10 / ((time.perf_counter() - t1) * 1e9)
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.sweeps(sp, 1.0 / p.T, p.seed, p.stream_id, 10, 2, record=True)
        paper_one = p.L * p.L * 2 / ((time.perf_counter() - t1) * 1e9)
    finally:
        oracle.set_threads(threads)
    out = {"value": ups, "unit": "spin updates/ns", "cores": threads, "kind": "oracle",
           "sample": sample, "cpu_model": cpu_model()}
    if one is not None:
        out["one_core"] = one
    out.update({
            "paper_point": {"workload": "%dx%d, T = 0.99 T_C, 10 sweeps (all cores), 2 sweeps "
                                        "(one core)" % (p.L, p.L),
                            "value": round(paper_all, 4), "value_1core": round(paper_one, 4)}})
    return out


def time_plain(torch, ising, dev, stream, w, steps, warmup, check=True):
    """w.sweeps sweeps per step with per-sweep E/M on a fresh lattice: warm-up
    steps, then `steps` steps timed with HIP events on the lattice's stream.
    Returns (ms for the timed steps, wall seconds, the lattice, its E/M buffer)."""
    lat = ising.Lattice(w.L, seed=w.seed, stream_id=w.stream_id, init=w.init, beta=1.0 / w.T,
                        device=dev, stream=stream)
    EM = torch.empty((w.sweeps, 2), dtype=torch.int64, device=dev)
    for _ in range(warmup):
        lat.sweep(w.sweeps, EM)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        lat.sweep(w.sweeps, EM)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = start.elapsed_time(stop)
    if check:
        # the last step's final (E, M) against an independent recount
        assert tuple(EM[-1].cpu().tolist()) == lat.measure(), "fused E/M disagrees with a recount"
    return ms, wall, lat, EM


def bench_configs(torch, ising, dev, stream, head):
    """The other plain configurations, each on a fresh lattice."""
    out = {}
    others = [(workloads.HUGE_T3, 2, 1), (workloads.LARGE, 5, 1), (workloads.SMALL, 20, 2)]
    for w, steps, warmup in others:
        if w == head:
            continue
        print("bench: plain %s (%d steps)" % (w.name, steps), file=sys.stderr, flush=True)
        ms, _, lat, EM = time_plain(torch, ising, dev, stream, w, steps, warmup)
        N = w.L * w.L
        out[w.name] = {"value": round(N * w.sweeps * steps / (ms * 1e6), 2),
                       "unit": "spin updates/ns",
                       "workload": "%dx%d, T=%r, %s start, %d sweeps per run with per-sweep "
                                   "int64 E/M" % (w.L, w.L, w.T,
                                                  ["cold +1", "cold -1", "hot"][w.init],
                                                  w.sweeps),
                       "ms_per_run": round(ms / steps, 3),
                       "us_per_sweep": round(ms * 1e3 / (steps * w.sweeps), 3),
                       "form": plain_kernel(ising, w.L, ising.tuning_lookup(w.L))}
        del lat, EM
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only (each lattice is held whole by one "
              "MI355X); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1007_3726_amd import ising

    w = {"large": workloads.LARGE, "huge-T2": workloads.HUGE_T2, "huge-T3": workloads.HUGE_T3,
         "small": workloads.SMALL, "paper-4096": workloads.PAPER_POINT}[args.workload]
    if args.sweeps is not None:
        import dataclasses
        w = dataclasses.replace(w, sweeps=args.sweeps)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    # the headline runs the library's built-in launch shape; the autotuner's
    # pick for this side is timed and reported beside it, then removed again
    autotuned = None
    if not args.no_autotune:
        t_at = time.perf_counter()
        pick = ising.autotune(w.L, trial_sweeps=max(2, min(100, int(2.7e10 / (w.L * w.L)))),
                              device=dev, stream=stream)
        autotuned = {"form": ["tile", "strip"][pick["form"]], "rpw": pick["rpw"],
                     "max_blocks": pick["max_blocks"],
                     "lds_resident_bytes": pick["small_lds_bytes"],
                     "updates_per_ns": round(pick["updates_per_ns"], 1),
                     "seconds": round(time.perf_counter() - t_at, 3)}
        ising.tuning_clear()
        torch.cuda.empty_cache()
    tuned = ising.tuning_lookup(w.L)
    kernel = plain_kernel(ising, w.L, tuned)
    print("bench: %s L=%d T=%r sweeps/step=%d warmup=%d steps=%d"
          % (w.name, w.L, w.T, w.sweeps, args.warmup, args.steps), file=sys.stderr, flush=True)
    ms, wall, lat, EM = time_plain(torch, ising, dev, stream, w, args.steps, args.warmup)
    N = w.L * w.L
    updates = N * w.sweeps * args.steps
    value = updates / (ms * 1e6)
    launches = 2 * w.sweeps * args.steps
    launch_us = ms * 1e3 / launches
    ops_per_launch = ALU_OPS_PER_UPDATE * N / 2
    achieved = ops_per_launch / (launch_us * 1e-6)
    del lat, EM
    torch.cuda.empty_cache()
    start_kind = ["cold +1", "cold -1", "hot"][w.init]
    result = {
        "metric": "spin updates/ns (packed checkerboard), batched vs plain; p50/p99 solve latency",
        "value": round(value, 2),
        "unit": "spin updates/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "plain %dx%d periodic lattice (%.2g spins, %.1f GiB packed), "
                               "T=%r, %s start from seed %d, %d sweeps/step, per-sweep int64 "
                               "E/M" % (w.L, w.L, float(N), ising.ising_lattice_bytes(w.L) / 2**30,
                                        w.T, start_kind, w.seed, w.sweeps),
                   "L": w.L, "T": w.T, "sweeps_per_step": w.sweeps, "form": "plain"},
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 3),
                     "peak": round(VALU_PEAK_LANE_OPS / 1e12, 3), "unit": "Tops/s",
                     "frac": round(achieved / VALU_PEAK_LANE_OPS, 4),
                     "traffic": profiled_traffic(kernel, w.L),
                     "algorithmic_bytes_per_launch": 3 * N // 16,
                     "kernel": kernel, "avg_launch_us": round(launch_us, 3),
                     "ops_per_update": ALU_OPS_PER_UPDATE},
        "wall_s": round(wall, 3),
        "shape": {"form": ["tile", "strip"][tuned["form"]], "rpw": tuned["rpw"],
                  "max_blocks": tuned["max_blocks"],
                  "lds_resident_bytes": tuned["small_lds_bytes"]},
        "autotuner_pick": autotuned,
    }
    if not args.no_configs:
        result["configs"] = bench_configs(torch, ising, dev, stream, w)
    side = workloads.LARGE if (w.L > 65536 and args.side_workload == "large") else w
    side_steps = max(1, min(args.steps, 3))
    if not args.no_lcg:
        print("bench: %s with the paper's LCG random numbers" % side.name, file=sys.stderr,
              flush=True)
        result["lcg"] = bench_lcg(torch, ising, dev, side, side_steps)
    if not args.no_pool:
        print("bench: %s with Boltzmann-pattern pools" % side.name, file=sys.stderr, flush=True)
        result["pool"] = bench_pool(torch, ising, dev, side, side_steps)
    if not args.no_strip:
        print("bench: one GPU's share of the row-strip decomposition", file=sys.stderr,
              flush=True)
        result["strip_share"] = bench_strip_share(torch, ising, dev)
    if not args.no_table2:
        print("bench: the paper's benchmark point (Table 2) with every variant", file=sys.stderr,
              flush=True)
        result["table2"] = bench_table2(torch, ising, dev)
    if args.copy_calibration:
        # a plain copy of known size: 1 GiB read + 1 GiB written
        src = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = 1 << 30
        del src, dst
    if not args.no_batched:
        print("bench: batched FSS grid (%d sweeps)" % args.batched_sweeps, file=sys.stderr,
              flush=True)
        if args.batched_shape:
            ising.batch_tuning_set(*[int(v) for v in args.batched_shape.split(",")])
        result["batched"] = bench_batched(torch, ising, dev, args.batched_sweeps,
                                          autotune=not (args.no_autotune or args.batched_shape))
        # the pick is the grid's: later legs (the server) keep the built-in shape
        ising.batch_tuning_clear()
        if not args.no_fss_proof:
            print("bench: FSS proof of concept (small lattices, long runs)", file=sys.stderr,
                  flush=True)
            result["fss_proof"] = bench_fss_proof(torch, ising, dev)
        torch.cuda.empty_cache()
    if not args.no_served:
        print("bench: served stream (%d requests)" % args.served_requests, file=sys.stderr,
              flush=True)
        result["served"] = bench_served(torch, ising, dev, args.served_requests,
                                        args.served_arena_gib, args.served_quantum,
                                        args.plain_fifo_requests, value, args.served_capacity)
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_sweeps, args.cpu_rows)
    if not args.no_cpu_msc:
        print("bench: multi-spin-coded CPU baseline (%s)" % side.name, file=sys.stderr,
              flush=True)
        result["cpu_msc"] = cpu_msc(side, result["configs"][side.name]["value"]
                                    if side is not w and "configs" in result else value)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
