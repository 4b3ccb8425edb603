"""Seeded synthetic workloads (inputs only; no Ising arithmetic here).

Shared by the tests, the benchmark and the smoke check so that the oracle
and the HIP path receive identical inputs.  Nothing in this module computes
any part of the method: it only names lattice sizes, temperatures, seeds,
stream ids, sweep counts and request arrival streams.

The workloads follow the paper's problem statement (an L x L periodic
lattice at temperature T, checkerboard Metropolis sweeps, magnetisation and
Binder cumulant; sections 3-5) at the sizes of the benchmark configurations.
"""
from dataclasses import dataclass
from typing import List

import numpy as np

INIT_COLD_UP = 0
INIT_COLD_DOWN = 1
INIT_HOT = 2

# Critical temperature as quoted in section 1 of the paper.
T_C_PAPER = 2.269185


@dataclass(frozen=True)
class Plain:
    name: str
    L: int
    T: float
    init: int
    seed: int
    stream_id: int
    sweeps: int


# Small plain lattice: 64 x 64, T = 2.269, hot start from seed 1, 1000 sweeps.
SMALL = Plain("plain-64", 64, 2.269, INIT_HOT, 1, 0, 1000)
# Plain lattice of the headline metric: 16384 x 16384, T = 2.269185, all +1, 2000 sweeps.
LARGE = Plain("plain-16384", 16384, T_C_PAPER, INIT_COLD_UP, 1, 0, 2000)
# HBM-resident lattice: 262144 x 262144 (8 GiB packed), hot start from seed 7, 100 sweeps.
HUGE_T2 = Plain("plain-262144-T2", 262144, 2.0, INIT_HOT, 7, 0, 100)
HUGE_T3 = Plain("plain-262144-T3", 262144, 3.0, INIT_HOT, 7, 0, 100)
# The paper's own benchmark point: 4096 x 4096 at 0.99 T_C (section 5.4).
PAPER_POINT = Plain("plain-4096-0.99Tc", 4096, 0.99 * T_C_PAPER, INIT_HOT, 1, 0, 200)

# Finite-size-scaling grid: L in {64..4096} x 32 temperatures in [2.20, 2.34].
FSS_SIZES = [64, 128, 256, 512, 1024, 2048, 4096]
FSS_TEMPS = [float(t) for t in np.linspace(2.20, 2.34, 32)]
FSS_SWEEPS = 10_000
FSS_DISCARD = 2_000


@dataclass(frozen=True)
class Lattice:
    L: int
    T: float
    init: int
    seed: int
    stream_id: int


def fss_grid(sizes=None, temps=None) -> List[Lattice]:
    """The 224-lattice grid; stream_id = 32 * size_index + T_index, seed 1, hot start."""
    sizes = FSS_SIZES if sizes is None else sizes
    temps = FSS_TEMPS if temps is None else temps
    out = []
    for si, L in enumerate(sizes):
        for ti, T in enumerate(temps):
            out.append(Lattice(L, T, INIT_HOT, 1, 32 * si + ti))
    return out


@dataclass(frozen=True)
class Request:
    index: int
    arrival: float  # seconds after the stream starts
    L: int
    T: float
    sweeps: int
    seed: int
    stream_id: int
    init: int


def served_stream(n: int = 2000, rate: float = 7.0, rng_seed: int = 20100707,
                  L_min: int = 32, L_max: int = 8192, sw_min: int = 1000,
                  sw_max: int = 100_000) -> List[Request]:
    """Poisson arrivals at `rate` per second; L log-uniform in [L_min, L_max]
    rounded to a multiple of 32; T uniform in [1.5, 3.5]; sweeps log-uniform
    in [sw_min, sw_max]; seed 1000 + i; hot start."""
    rng = np.random.default_rng(rng_seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    Ls = np.exp(rng.uniform(np.log(L_min), np.log(L_max), size=n))
    Ls = np.clip(32 * np.round(Ls / 32), 32, L_max).astype(np.int64)
    Ts = rng.uniform(1.5, 3.5, size=n)
    sw = np.round(np.exp(rng.uniform(np.log(sw_min), np.log(sw_max), size=n))).astype(np.int64)
    return [Request(i, float(arrivals[i]), int(Ls[i]), float(Ts[i]), int(sw[i]), 1000 + i, 0,
                    INIT_HOT) for i in range(n)]
