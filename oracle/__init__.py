"""CPU oracle for the checkerboard Metropolis sweep of the 2D Ising model.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(``paper_1007_3726_amd``) never imports it and shares no code with it.

Thin ctypes wrapper over ``ising_oracle.c``; every function below forwards to
the C routine of the same role, whose comments cite the paper's sections and
equations.
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    """Load (building first if missing or stale) the oracle shared library."""
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        u32, i32, i64, u64 = ctypes.c_uint32, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
        p8 = ctypes.POINTER(ctypes.c_int8)
        p64 = ctypes.POINTER(ctypes.c_int64)
        pu32 = ctypes.POINTER(ctypes.c_uint32)
        L.oracle_philox4x32_10.argtypes = [pu32, pu32, pu32]
        L.oracle_philox4x32_10.restype = None
        L.oracle_threshold.argtypes = [ctypes.c_double, i32]
        L.oracle_threshold.restype = u32
        L.oracle_uniform.argtypes = [u64, u32, u32, u32, i64, i64, i64]
        L.oracle_uniform.restype = u32
        L.oracle_accept.argtypes = [i32, i32, i32, i32, i32, u32, u32, u32]
        L.oracle_accept.restype = i32
        L.oracle_init.argtypes = [i64, u64, u32, i32, p8]
        L.oracle_init.restype = None
        L.oracle_measure.argtypes = [i64, p8, p64, p64]
        L.oracle_measure.restype = None
        L.oracle_sweeps.argtypes = [i64, u32, u32, u64, u32, u32, i64, p8, p64]
        L.oracle_sweeps.restype = None
        L.oracle_window.argtypes = [i64, u32, u32, u64, u32, i32, u32, i64, i64, i64, i64, i64, p8]
        L.oracle_window.restype = i32
        pu32w = ctypes.POINTER(ctypes.c_uint32)
        L.oracle_lcg_threshold.argtypes = [ctypes.c_double, i32]
        L.oracle_lcg_threshold.restype = u32
        L.oracle_lcg_seed.argtypes = [i64, u64, pu32w]
        L.oracle_lcg_seed.restype = None
        L.oracle_lcg_sweeps.argtypes = [i64, u32, u32, i64, p8, pu32w, p64]
        L.oracle_lcg_sweeps.restype = None
        pu64 = ctypes.POINTER(ctypes.c_uint64)
        L.oracle_pool_fill.argtypes = [u64, u32, u32, u32, i32, pu64, pu64]
        L.oracle_pool_fill.restype = None
        L.oracle_pool_address.argtypes = [u64, u32, u32, i32, i32, i32, u64]
        L.oracle_pool_address.restype = u32
        L.oracle_pool_sweeps.argtypes = [i64, u32, u32, u64, u32, u32, i64, i32, i32, p8, p64]
        L.oracle_pool_sweeps.restype = i32
        L.oracle_band_em.argtypes = [i64, u32, u32, u64, u32, i32, u32, i64, i64, i64, p64]
        L.oracle_band_em.restype = i32
        L.oracle_pool_window.argtypes = [i64, u64, u32, i32, u32, i64, i32, i32, pu64, pu64,
                                         i64, i64, i64, i64, p8]
        L.oracle_pool_window.restype = i32
        L.oracle_lcg_window.argtypes = [i64, u32, u32, u64, u32, i32, i64, i64, i64, i64, i64,
                                        p8]
        L.oracle_lcg_window.restype = i32
        L.oracle_pool_band_em.argtypes = [i64, u64, u32, i32, u32, i64, i32, i32, pu64, pu64,
                                          i64, i64, p64]
        L.oracle_pool_band_em.restype = i32
        L.oracle_lcg_band_em.argtypes = [i64, u32, u32, u64, u32, i32, i64, i64, i64, p64]
        L.oracle_lcg_band_em.restype = i32
        L.oracle_get_threads.argtypes = []
        L.oracle_get_threads.restype = i32
        L.oracle_set_threads.argtypes = [i32]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def _p8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def philox4x32_10(ctr, key):
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return [int(o[i]) for i in range(4)]


def check_beta(beta: float) -> None:
    if math.isnan(beta) or beta < 0:
        raise ValueError("beta must be >= 0 (or +inf)")


def thresholds(beta: float):
    """(t4, t8): integer Metropolis thresholds for dE = 4 and dE = 8."""
    check_beta(beta)
    return int(lib().oracle_threshold(beta, 4)), int(lib().oracle_threshold(beta, 8))


def uniform(seed, stream_id, phase, t, L, x, y) -> int:
    return int(lib().oracle_uniform(seed, stream_id, phase, t, L, x, y))


def accept(s, n1, n2, n3, n4, u, t4, t8) -> int:
    return int(lib().oracle_accept(s, n1, n2, n3, n4, u, t4, t8))


def init(L: int, seed: int, stream_id: int, init_kind: int) -> np.ndarray:
    s = np.empty((L, L), dtype=np.int8)
    lib().oracle_init(L, seed, stream_id, init_kind, _p8(s))
    return s


def measure(s: np.ndarray):
    s = np.ascontiguousarray(s, dtype=np.int8)
    E = ctypes.c_int64()
    M = ctypes.c_int64()
    lib().oracle_measure(s.shape[0], _p8(s), ctypes.byref(E), ctypes.byref(M))
    return int(E.value), int(M.value)


def sweeps(s: np.ndarray, beta: float, seed: int, stream_id: int, t0: int, n: int,
           record: bool = True):
    """Run n sweeps in place on int8 spins s (L x L); returns EM[n, 2] or None."""
    assert s.dtype == np.int8 and s.flags.c_contiguous and s.shape[0] == s.shape[1]
    t4, t8 = thresholds(beta)
    EM = np.zeros((n, 2), dtype=np.int64) if record else None
    lib().oracle_sweeps(s.shape[0], t4, t8, seed, stream_id, t0, n, _p8(s),
                        _p64(EM) if record else None)
    return EM


def run(L: int, beta: float, seed: int, stream_id: int, init_kind: int, n: int):
    """Fresh lattice, n sweeps from t = 0: returns (spins, EM[n, 2])."""
    s = init(L, seed, stream_id, init_kind)
    EM = sweeps(s, beta, seed, stream_id, 0, n)
    return s, EM


def window(L, beta, seed, stream_id, init_kind, t0, n, x0, y0, w, h) -> np.ndarray:
    """Exact w x h window at (x0, y0) after n sweeps from a fresh init (light cone)."""
    t4, t8 = thresholds(beta)
    out = np.empty((h, w), dtype=np.int8)
    rc = lib().oracle_window(L, t4, t8, seed, stream_id, init_kind, t0, n, x0, y0, w, h, _p8(out))
    if rc != 0:
        raise ValueError("window plus light-cone margin does not fit in the lattice")
    return out


def band_em(L, beta, seed, stream_id, init_kind, t0, n, y0, h) -> np.ndarray:
    """The rows [y0, y0 + h)'s shares of (E, M) after each of n sweeps from a
    fresh init (light cone over full rows): int64 array [n, 2]."""
    t4, t8 = thresholds(beta)
    EM = np.zeros((n, 2), dtype=np.int64)
    rc = lib().oracle_band_em(L, t4, t8, seed, stream_id, init_kind, t0, n, y0, h, _p64(EM))
    if rc != 0:
        raise ValueError("band plus light-cone margin does not fit in the lattice")
    return EM


def lattice_em_by_bands(L, beta, seed, stream_id, init_kind, n, band_rows, progress=None):
    """Whole-lattice (E, M) after each of n sweeps from a fresh init, summed
    over bands of at most band_rows rows (memory ~ (band_rows + 4n + 2) L
    bytes instead of L^2): int64 array [n, 2]."""
    total = np.zeros((n, 2), dtype=np.int64)
    y0 = 0
    while y0 < L:
        h = min(band_rows, L - y0)
        total += band_em(L, beta, seed, stream_id, init_kind, 0, n, y0, h)
        y0 += h
        if progress is not None:
            progress(y0)
    return total


def lcg_thresholds(beta: float):
    """(t4', t8') of the per-thread LCG dynamics: min(floor(exp(-beta dE) 2^31), 2^31)."""
    check_beta(beta)
    return (int(lib().oracle_lcg_threshold(beta, 4)), int(lib().oracle_lcg_threshold(beta, 8)))


def lcg_seed(L: int, seed: int) -> np.ndarray:
    """Thread seeds of Eq. (7): uint32 array (2, L, W), state[c, y, w]."""
    W = (L // 2 + 63) // 64
    st = np.empty((2, L, W), dtype=np.uint32)
    lib().oracle_lcg_seed(L, seed, st.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return st


def lcg_sweeps(s: np.ndarray, beta: float, state: np.ndarray, n: int, record: bool = True):
    """n sweeps of the per-thread-LCG dynamics in place (spins and states);
    returns EM[n, 2] (or None)."""
    L = s.shape[0]
    assert s.dtype == np.int8 and s.flags.c_contiguous
    assert state.dtype == np.uint32 and state.flags.c_contiguous
    t4, t8 = lcg_thresholds(beta)
    EM = np.empty((n, 2), dtype=np.int64) if record else None
    lib().oracle_lcg_sweeps(L, t4, t8, n, _p8(s), state.ctypes.data_as(
        ctypes.POINTER(ctypes.c_uint32)), _p64(EM) if record else None)
    return EM


def pool_fill(beta: float, seed: int, stream_id: int, m: int):
    """Boltzmann-pattern pool of 2^m patterns for beta: (exp4, exp8), each a
    uint64 array whose bit b of entry p is that bit of pattern p."""
    t4, t8 = thresholds(beta)
    e4 = np.empty(1 << m, dtype=np.uint64)
    e8 = np.empty(1 << m, dtype=np.uint64)
    pu64 = ctypes.POINTER(ctypes.c_uint64)
    lib().oracle_pool_fill(seed, stream_id, t4, t8, m, e4.ctypes.data_as(pu64),
                           e8.ctypes.data_as(pu64))
    return e4, e8


def pool_address(seed: int, stream_id: int, t: int, colour: int, m: int, linear: bool,
                 j: int) -> int:
    """Pool pattern read by word j (= y W + w) in sweep t, colour `colour`."""
    return int(lib().oracle_pool_address(seed, stream_id, t, colour, m, 1 if linear else 0, j))


def pool_sweeps(s: np.ndarray, beta: float, seed: int, stream_id: int, t0: int, n: int, m: int,
                linear: bool, record: bool = True):
    """n sweeps in place with a pool of 2^m Boltzmann patterns (drawn for
    beta); linear: one address per 256-word group.  Returns EM[n, 2] or None."""
    assert s.dtype == np.int8 and s.flags.c_contiguous and s.shape[0] == s.shape[1]
    t4, t8 = thresholds(beta)
    EM = np.zeros((n, 2), dtype=np.int64) if record else None
    rc = lib().oracle_pool_sweeps(s.shape[0], t4, t8, seed, stream_id, t0, n, m,
                                  1 if linear else 0, _p8(s), _p64(EM) if record else None)
    if rc != 0:
        raise ValueError("bad pool size")
    return EM


def pool_window(L, beta, seed, stream_id, init_kind, t0, n, m, linear, x0, y0, w, h,
                pool=None) -> np.ndarray:
    """Exact w x h window at (x0, y0) after n sweeps (from sweep counter t0,
    fresh init) of the pattern-pool dynamics, by the light cone.  pool: the
    (exp4, exp8) arrays of pool_fill for the same beta, seed and stream id
    (filled here when None)."""
    e4, e8 = pool if pool is not None else pool_fill(beta, seed, stream_id, m)
    assert e4.dtype == np.uint64 and e8.dtype == np.uint64 and len(e4) == len(e8) == 1 << m
    out = np.empty((h, w), dtype=np.int8)
    pu64 = ctypes.POINTER(ctypes.c_uint64)
    rc = lib().oracle_pool_window(L, seed, stream_id, init_kind, t0, n, m, 1 if linear else 0,
                                  e4.ctypes.data_as(pu64), e8.ctypes.data_as(pu64), x0, y0, w,
                                  h, _p8(out))
    if rc != 0:
        raise ValueError("window plus light-cone margin does not fit in the lattice")
    return out


def lcg_window(L, beta, seed, stream_id, init_kind, n, x0, y0, w, h) -> np.ndarray:
    """Exact w x h window at (x0, y0) after n sweeps of the per-thread-LCG
    dynamics from a fresh init and the thread seeds of lcg_seed(L, seed)."""
    t4, t8 = lcg_thresholds(beta)
    out = np.empty((h, w), dtype=np.int8)
    rc = lib().oracle_lcg_window(L, t4, t8, seed, stream_id, init_kind, n, x0, y0, w, h,
                                 _p8(out))
    if rc != 0:
        raise ValueError("window plus light-cone margin does not fit in the lattice")
    return out


def lcg_band_em(L, beta, seed, stream_id, init_kind, n, y0, h) -> np.ndarray:
    """Rows [y0, y0 + h)'s shares of (E, M) after each of n sweeps of the
    per-thread-LCG dynamics (light cone over full rows): int64 [n, 2]."""
    t4, t8 = lcg_thresholds(beta)
    EM = np.zeros((n, 2), dtype=np.int64)
    rc = lib().oracle_lcg_band_em(L, t4, t8, seed, stream_id, init_kind, n, y0, h, _p64(EM))
    if rc != 0:
        raise ValueError("band plus light-cone margin does not fit in the lattice")
    return EM


def pool_band_em(L, beta, seed, stream_id, init_kind, t0, n, m, linear, y0, h,
                 pool=None) -> np.ndarray:
    """Rows [y0, y0 + h)'s shares of (E, M) after each of n sweeps of the
    pattern-pool dynamics (light cone over full rows): int64 [n, 2]."""
    e4, e8 = pool if pool is not None else pool_fill(beta, seed, stream_id, m)
    EM = np.zeros((n, 2), dtype=np.int64)
    pu64 = ctypes.POINTER(ctypes.c_uint64)
    rc = lib().oracle_pool_band_em(L, seed, stream_id, init_kind, t0, n, m, 1 if linear else 0,
                                   e4.ctypes.data_as(pu64), e8.ctypes.data_as(pu64), y0, h,
                                   _p64(EM))
    if rc != 0:
        raise ValueError("band plus light-cone margin does not fit in the lattice")
    return EM


def set_threads(n: int) -> None:
    lib().oracle_set_threads(n)


def get_threads() -> int:
    return int(lib().oracle_get_threads())
