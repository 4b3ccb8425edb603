"""Multi-spin-coded CPU baseline of the checkerboard Metropolis sweep.

The paper states its GPU speed-ups against an optimised multi-spin-coded CPU
program (sections 4 and 5.4).  ``msc_cpu.c`` is such a program for the same
Markov chain as the GPU library (same layout, keying and acceptance rule),
so the benchmark can report the GPU against a fair CPU figure on the same
host.  It is a measurement baseline: the GPU library never uses it, and it
shares no code with the GPU library or the oracle.
"""
import ctypes

import numpy as np

from . import build as _build

_lib = None


def lib():
    """Load (building first if missing or stale) the baseline library."""
    global _lib
    if _lib is None:
        L = ctypes.CDLL(_build.build(force=False))
        i32, i64, u32, u64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
        pu64 = ctypes.POINTER(ctypes.c_uint64)
        p64 = ctypes.POINTER(ctypes.c_int64)
        p8 = ctypes.POINTER(ctypes.c_int8)
        L.msc_bytes.argtypes = [i64]
        L.msc_bytes.restype = i64
        L.msc_vector_available.argtypes = []
        L.msc_vector_available.restype = i32
        L.msc_init.argtypes = [pu64, i64, u64, u32, i32, i32]
        L.msc_init.restype = i32
        L.msc_sweeps.argtypes = [pu64, i64, u64, u32, ctypes.c_double, u32, i64, p64, i32]
        L.msc_sweeps.restype = i32
        L.msc_get_spins.argtypes = [pu64, i64, p8]
        L.msc_get_spins.restype = None
        L.msc_scalar_only.argtypes = [i32]
        L.msc_pool_fill.argtypes = [pu64, i32, u64, u32, ctypes.c_double, i32]
        L.msc_pool_fill.restype = i32
        L.msc_pool_sweeps.argtypes = [pu64, i64, u64, u32, pu64, i32, i32, u32, i64, p64, i32]
        L.msc_pool_sweeps.restype = i32
        L.msc_word_masks.argtypes = [i64, u64, u32, i64, i64, u32, u32, u32, u32, pu64]
        L.msc_word_masks.restype = None
        L.msc_scalar_only.restype = None
        _lib = L
    return _lib


def vector_available() -> bool:
    return bool(lib().msc_vector_available())


def scalar_only(on: bool) -> None:
    """Force the scalar Philox (tests of both code paths)."""
    lib().msc_scalar_only(1 if on else 0)


def word_masks(L, seed, stream_id, y, w, t, phase, ta, tb):
    """(mask of [u < ta], mask of [u < tb]) over the sites of word (y, w)."""
    out = np.zeros(2, dtype=np.uint64)
    lib().msc_word_masks(L, seed, stream_id, y, w, t, phase, ta, tb,
                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return int(out[0]), int(out[1])


class Lattice:
    """An L x L lattice in host memory (two colour planes of 64-spin words)."""

    def __init__(self, L: int, seed: int = 1, stream_id: int = 0, init: int = 2,
                 threads: int = 0):
        nbytes = lib().msc_bytes(L)
        if nbytes <= 0:
            raise ValueError("L must be even and >= 4")
        self.L, self.seed, self.stream_id, self.threads = L, seed, stream_id, threads
        self.planes = np.zeros(nbytes // 8, dtype=np.uint64)
        self.t = 0
        if lib().msc_init(self._p(), L, seed, stream_id, init, threads) != 0:
            raise ValueError("bad init")

    def _p(self):
        return self.planes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))

    def sweeps(self, beta: float, n: int, record: bool = True):
        """n sweeps at inverse temperature beta; (n, 2) int64 (E, M) per sweep."""
        EM = np.zeros((n, 2), dtype=np.int64) if record else None
        p = EM.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if record else None
        if lib().msc_sweeps(self._p(), self.L, self.seed, self.stream_id, beta, self.t, n, p,
                            self.threads) != 0:
            raise ValueError("bad arguments")
        self.t += n
        return EM

    def use_pool(self, beta: float, log2_patterns: int = 22, linear: bool = False):
        """Switch to the Boltzmann-pattern-pool dynamics (the paper's CPU
        scheme) with a pool drawn for beta; sweeps() then reads it."""
        self.pool = np.zeros(2 << log2_patterns, dtype=np.uint64)
        pu64 = ctypes.POINTER(ctypes.c_uint64)
        if lib().msc_pool_fill(self.pool.ctypes.data_as(pu64), log2_patterns, self.seed,
                               self.stream_id, beta, self.threads) != 0:
            raise ValueError("bad pool arguments")
        self.pool_m, self.pool_linear, self.pool_beta = log2_patterns, linear, beta

    def pool_sweeps(self, n: int, record: bool = True):
        """n sweeps of the pool dynamics (use_pool first); (n, 2) int64 (E, M)."""
        EM = np.zeros((n, 2), dtype=np.int64) if record else None
        p = EM.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if record else None
        pu64 = ctypes.POINTER(ctypes.c_uint64)
        if lib().msc_pool_sweeps(self._p(), self.L, self.seed, self.stream_id,
                                 self.pool.ctypes.data_as(pu64), self.pool_m,
                                 1 if self.pool_linear else 0, self.t, n, p, self.threads) != 0:
            raise ValueError("bad arguments")
        self.t += n
        return EM

    def spins(self) -> np.ndarray:
        out = np.empty((self.L, self.L), dtype=np.int8)
        lib().msc_get_spins(self._p(), self.L, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
        return out
