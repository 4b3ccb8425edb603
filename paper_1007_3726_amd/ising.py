"""ctypes binding of the C ABI in include/ising.h (argument marshalling only).

Every computation runs in libising.so (HIP kernels for gfx950).  PyTorch is
used only to allocate device memory (uint8 tensors) and to name HIP streams.
If the library is missing this module raises: there is no CPU fallback.
"""
import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libising.so")

ISING_OK = 0
ISING_AGAIN = 1
ISING_EINVAL = -1
ISING_ENOMEM = -2
ISING_EDEVICE = -3
ISING_ENOTFOUND = -4
ISING_ERANGE = -5
ISING_FORM_TILE = 0
ISING_FORM_STRIP = 1
ISING_RNG_PHILOX = 0
ISING_RNG_LCG = 1
ISING_RNG_POOL = 2
ISING_RNG_POOL_LINEAR = 3

INIT_COLD_UP = 0
INIT_COLD_DOWN = 1
INIT_HOT = 2

REQ_RECORD_SERIES = 1
REQ_RETURN_SPINS = 2


class IsingError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("ising error %d: %s" % (code, msg))
        self.code = code


class ising_request(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int64), ("beta", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("stream_id", ctypes.c_uint32), ("init", ctypes.c_int32),
                ("n_sweeps", ctypes.c_int64), ("n_discard", ctypes.c_int64),
                ("flags", ctypes.c_uint32), ("EM_series", ctypes.POINTER(ctypes.c_int64)),
                ("spins_out", ctypes.POINTER(ctypes.c_int8))]


class ising_tuning(ctypes.Structure):
    _fields_ = [("L_min", ctypes.c_int64), ("L_max", ctypes.c_int64), ("form", ctypes.c_int32),
                ("rpw", ctypes.c_int32), ("max_blocks", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("small_lds_bytes", ctypes.c_int64),
                ("updates_per_ns", ctypes.c_double)]


class ising_batch_tuning(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("rpw_max", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32), ("graph_chunk", ctypes.c_int32),
                ("updates_per_ns", ctypes.c_double), ("default_updates_per_ns", ctypes.c_double),
                ("packed_updates_per_ns", ctypes.c_double)]


class ising_result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("E_final", ctypes.c_int64), ("M_final", ctypes.c_int64),
                ("sweeps_done", ctypes.c_uint64), ("sum_M2", ctypes.c_double),
                ("sum_M4", ctypes.c_double), ("n_kept", ctypes.c_int64),
                ("t_arrive", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


_lib = None


def lib():
    """Load libising.so (built by paper_1007_3726_amd/build.py); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libising.so is not built (run __graft_entry__.build()); "
                           "there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                              ctypes.c_uint64)
    P = ctypes.POINTER
    sig = {
        "ising_last_error": ([], ctypes.c_char_p),
        "ising_version": ([], ctypes.c_char_p),
        "ising_lattice_bytes": ([i64], ctypes.c_size_t),
        "ising_create": ([i64, u64, u32, i32, vp, ctypes.c_size_t, vp, P(vp)], i32),
        "ising_destroy": ([vp], i32),
        "ising_set_beta": ([vp, ctypes.c_double], i32),
        "ising_get_thresholds": ([vp, P(u32)], i32),
        "ising_sweep": ([vp, i64, vp], i32),
        "ising_measure": ([vp, P(i64), P(i64)], i32),
        "ising_get_spins": ([vp, vp], i32),
        "ising_set_spins": ([vp, vp], i32),
        "ising_get_window": ([vp, i64, i64, i64, i64, vp], i32),
        "ising_get_sweep": ([vp, P(u64)], i32),
        "ising_set_sweep": ([vp, u64], i32),
        "ising_get_info": ([vp, P(i64), P(i64), P(vp)], i32),
        "ising_multi_sweep_work_bytes": ([P(vp), i32, P(ctypes.c_size_t)], i32),
        "ising_multi_sweep_static": ([P(vp), i32, i64, P(vp)], i32),
        "ising_multi_sweep": ([P(vp), i32, i64, P(vp), vp, ctypes.c_size_t], i32),
        "ising_multi_sweep_form": ([P(vp), i32, i64, P(vp), i32, i32, vp, ctypes.c_size_t],
                                   i32),
        "ising_batch_plan": ([P(i64), i32, i32, P(i32), P(i32), P(ctypes.c_double)], i32),
        "ising_autotune": ([i64, vp, ctypes.c_size_t, vp, i32, P(ising_tuning)], i32),
        "ising_tuning_set": ([P(ising_tuning), i32], i32),
        "ising_tuning_get": ([P(ising_tuning), i32, P(i32)], i32),
        "ising_tuning_clear": ([], i32),
        "ising_tuning_lookup": ([i64, P(ising_tuning)], i32),
        "ising_multi_autotune_bytes": ([P(vp), i32, i32, P(ctypes.c_size_t)], i32),
        "ising_multi_autotune": ([P(vp), i32, i32, vp, ctypes.c_size_t, P(ising_batch_tuning)],
                                 i32),
        "ising_batch_tuning_set": ([P(ising_batch_tuning)], i32),
        "ising_batch_tuning_get": ([P(ising_batch_tuning), P(i32)], i32),
        "ising_batch_tuning_clear": ([], i32),
        "ising_server_create": ([vp, ctypes.c_size_t, vp, i32, P(vp)], i32),
        "ising_batch_submit": ([vp, P(ising_request), i32, P(u64)], i32),
        "ising_server_step": ([vp], i32),
        "ising_poll": ([vp, u64, P(ising_result)], i32),
        "ising_server_inject_fault": ([vp, i64], i32),
        "ising_server_stats": ([vp, P(i64)], i32),
        "ising_server_destroy": ([vp], i32),
        "ising_series_moments": ([vp, i64, i64, P(ctypes.c_double), P(ctypes.c_double), P(i64)],
                                 i32),
        "ising_lcg_bytes": ([i64], ctypes.c_size_t),
        "ising_pool_bytes": ([i32], ctypes.c_size_t),
        "ising_debug_perturb": ([u32], i32),
        "ising_strip_bytes": ([i64, i64], ctypes.c_size_t),
        "ising_strip_create": ([i64, i64, i64, u64, u32, i32, vp, ctypes.c_size_t, vp, P(vp)],
                               i32),
        "ising_strip_destroy": ([vp], i32),
        "ising_strip_set_beta": ([vp, ctypes.c_double], i32),
        "ising_strip_step": ([vp, i32, u32, vp], i32),
        "ising_strip_exchange": ([P(vp), i32, i32], i32),
        "ising_strip_row": ([vp, i32, i32, P(vp), P(ctypes.c_size_t)], i32),
        "ising_strip_get_rows": ([vp, vp], i32),
        "ising_strip_combine": ([vp, i32, i64, i64, vp, vp], i32),
        "ising_set_rng": ([vp, i32, vp, ctypes.c_size_t], i32),
        "ising_reweight": ([i32, P(vp), P(i64), P(i64), P(ctypes.c_double), i32, P(i32),
                            P(ctypes.c_double), i32, vp, vp, vp, ctypes.c_size_t, vp], i32),
        "ising_reweight_work_bytes": ([i32, i32], ctypes.c_size_t),
        "ising_fss_moments": ([vp, i32, i32, P(i64), vp, vp, vp], i32),
        "ising_autocorr_time": ([vp, i64, ctypes.c_double, P(ctypes.c_double), P(i64)], i32),
        "ising_binder_crossing": ([vp, i32, vp, vp, vp, vp, i32, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return _lib


def check(code: int, ok=(ISING_OK,)) -> int:
    if code not in ok:
        raise IsingError(code, lib().ising_last_error().decode())
    return code


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def torch_uint32():
    """A 4-byte torch dtype for viewing uint32 buffers (bit pattern only)."""
    import torch
    return torch.int32


def _dev_alloc(nbytes: int, device):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------------------
# Module-level functions with the ABI's names
# ---------------------------------------------------------------------------
def ising_lattice_bytes(L: int) -> int:
    return int(lib().ising_lattice_bytes(L))


def ising_lcg_bytes(L: int) -> int:
    return int(lib().ising_lcg_bytes(L))


class StripSet:
    """A lattice split into row strips, each one GPU's share in a multi-GPU
    decomposition, all held here on one device: every colour step runs
    on each strip, then the halos of that colour are exchanged
    (ising_strip_exchange stands in for RCCL send/recv between GPUs)."""

    def __init__(self, L: int, nstrips: int, seed: int = 1, stream_id: int = 0,
                 init: int = INIT_HOT, beta: Optional[float] = None, rows=None,
                 device="cuda", stream=None):
        import torch
        if rows is None:
            base, extra = divmod(L, nstrips)
            rows = [base + (1 if k < extra else 0) for k in range(nstrips)]
        assert len(rows) == nstrips and sum(rows) == L
        self.L, self.rows, self.device = L, list(rows), device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.bufs, self.hs = [], []
        y0 = 0
        for r in rows:
            nbytes = int(lib().ising_strip_bytes(L, r))
            if nbytes == 0:
                raise IsingError(ISING_EINVAL, "unsupported strip shape L=%d rows=%d" % (L, r))
            buf = _dev_alloc(nbytes, device)
            h = ctypes.c_void_p()
            check(lib().ising_strip_create(L, y0, r, seed, stream_id, init, buf.data_ptr(), nbytes,
                                           _stream_ptr(self.stream), ctypes.byref(h)))
            self.bufs.append(buf)
            self.hs.append(h)
            y0 += r
        self._arr = (ctypes.c_void_p * nstrips)(*[h.value for h in self.hs])
        for c in (0, 1):
            check(lib().ising_strip_exchange(self._arr, nstrips, c))
        self.t = 0
        if beta is not None:
            self.set_beta(beta)

    def close(self):
        for h in self.hs:
            lib().ising_strip_destroy(h)
        self.hs = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_beta(self, beta: float):
        for h in self.hs:
            check(lib().ising_strip_set_beta(h, beta))

    def sweep_em(self, n: int):
        """n sweeps; returns the lattice's (E, M) after each sweep as a device
        int64 tensor (n, 2)."""
        import torch
        G = len(self.hs)
        counts = torch.empty((max(n, 1), G, 2), dtype=torch.int64, device=self.device)
        EM = torch.empty((max(n, 1), 2), dtype=torch.int64, device=self.device)
        for k in range(n):
            t = self.t + k
            for c in (0, 1):
                for s, h in enumerate(self.hs):
                    ptr = counts[k, s].data_ptr() if c == 1 else None
                    check(lib().ising_strip_step(h, c, t, ptr))
                check(lib().ising_strip_exchange(self._arr, G, c))
        check(lib().ising_strip_combine(counts.data_ptr(), G, n, self.L, EM.data_ptr(),
                                        _stream_ptr(self.stream)))
        self.t += n
        return EM[:n]

    def get_spins(self):
        import numpy as np
        out = np.empty((self.L, self.L), dtype=np.int8)
        y0 = 0
        for h, r in zip(self.hs, self.rows):
            part = np.empty((r, self.L), dtype=np.int8)
            check(lib().ising_strip_get_rows(h, part.ctypes.data))
            out[y0:y0 + r] = part
            y0 += r
        return out


def debug_perturb(seed: int) -> None:
    """Barrier-perturbation test hook (0: off): waves pause pseudo-randomly
    before the block barriers of the LDS-resident and packed kernels."""
    check(lib().ising_debug_perturb(seed))


def ising_pool_bytes(log2_patterns: int) -> int:
    return int(lib().ising_pool_bytes(log2_patterns))


def ising_version() -> str:
    return lib().ising_version().decode()


class Lattice:
    """One L x L lattice whose packed planes live in a torch uint8 tensor."""

    def __init__(self, L: int, seed: int = 1, stream_id: int = 0, init: int = INIT_HOT,
                 beta: Optional[float] = None, device="cuda", stream=None):
        import torch
        nbytes = ising_lattice_bytes(L)
        if nbytes == 0:
            raise IsingError(ISING_EINVAL, "invalid lattice side %r" % (L,))
        self.L = int(L)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.buf = _dev_alloc(nbytes, self.device)
        h = ctypes.c_void_p()
        check(lib().ising_create(self.L, seed & (2 ** 64 - 1), stream_id, init, self.buf.data_ptr(),
                                 nbytes, _stream_ptr(self.stream), ctypes.byref(h)))
        self.h = h
        if beta is not None:
            self.set_beta(beta)

    def close(self):
        if getattr(self, "h", None):
            lib().ising_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_beta(self, beta: float):
        check(lib().ising_set_beta(self.h, float(beta)))

    def use_lcg(self):
        """Switch to the paper's per-thread LCG dynamics (ising_set_rng); the
        state buffer is allocated here and seeded on the lattice's stream."""
        nbytes = ising_lcg_bytes(self.L)
        self.lcg_buf = _dev_alloc(max(nbytes, 4), self.device)
        check(lib().ising_set_rng(self.h, ISING_RNG_LCG, self.lcg_buf.data_ptr(), nbytes))

    def use_pool(self, log2_patterns: int = 22, linear: bool = False):
        """Switch to the Boltzmann-pattern-pool dynamics (ising_set_rng): a
        pool of 2^log2_patterns patterns, allocated here and drawn on the
        lattice's stream; linear reads one random start per 256 words."""
        nbytes = ising_pool_bytes(log2_patterns)
        self.pool_buf = _dev_alloc(max(nbytes, 16), self.device)
        kind = ISING_RNG_POOL_LINEAR if linear else ISING_RNG_POOL
        check(lib().ising_set_rng(self.h, kind, self.pool_buf.data_ptr(), nbytes))
        self.lcg_buf = None

    def use_philox(self):
        check(lib().ising_set_rng(self.h, ISING_RNG_PHILOX, None, 0))
        self.lcg_buf = None
        self.pool_buf = None

    def lcg_states(self):
        """Host copy of the LCG states as uint32 (2, L, W)."""
        import numpy as np
        W = (self.L // 2 + 63) // 64
        self.stream.synchronize()
        return self.lcg_buf.view(torch_uint32()).cpu().numpy().view(np.uint32).reshape(2, self.L, W)

    def thresholds(self):
        t = (ctypes.c_uint32 * 2)()
        check(lib().ising_get_thresholds(self.h, t))
        return int(t[0]), int(t[1])

    def sweep(self, n: int, EM=None):
        """Enqueue n sweeps; EM: None, or a device int64 tensor (n, 2) to fill."""
        ptr = None
        if EM is not None:
            assert EM.dtype.itemsize == 8 and EM.is_cuda and EM.numel() >= 2 * n
            assert EM.is_contiguous()
            ptr = EM.data_ptr()
        check(lib().ising_sweep(self.h, int(n), ptr))

    def sweep_em(self, n: int):
        """n sweeps; returns the (n, 2) int64 device tensor of (E, M) per sweep."""
        import torch
        EM = torch.empty((n, 2), dtype=torch.int64, device=self.device)
        self.sweep(n, EM)
        return EM

    def measure(self):
        E, M = ctypes.c_int64(), ctypes.c_int64()
        check(lib().ising_measure(self.h, ctypes.byref(E), ctypes.byref(M)))
        return int(E.value), int(M.value)

    def get_spins(self) -> np.ndarray:
        out = np.empty((self.L, self.L), dtype=np.int8)
        check(lib().ising_get_spins(self.h, out.ctypes.data))
        return out

    def set_spins(self, s: np.ndarray):
        s = np.ascontiguousarray(s, dtype=np.int8)
        assert s.shape == (self.L, self.L)
        check(lib().ising_set_spins(self.h, s.ctypes.data))

    def get_window(self, x0: int, y0: int, w: int, h: int) -> np.ndarray:
        out = np.empty((h, w), dtype=np.int8)
        check(lib().ising_get_window(self.h, x0, y0, w, h, out.ctypes.data))
        return out

    @property
    def sweep_count(self) -> int:
        t = ctypes.c_uint64()
        check(lib().ising_get_sweep(self.h, ctypes.byref(t)))
        return int(t.value)

    @sweep_count.setter
    def sweep_count(self, t: int):
        check(lib().ising_set_sweep(self.h, int(t)))

    def planes(self):
        """(L, W, device address) of the packed planes."""
        L, W, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_void_p()
        check(lib().ising_get_info(self.h, ctypes.byref(L), ctypes.byref(W), ctypes.byref(p)))
        return int(L.value), int(W.value), int(p.value or 0)


_TUNING_KEYS = ["L_min", "L_max", "form", "rpw", "max_blocks", "small_lds_bytes",
                "updates_per_ns"]


def autotune(L: int, trial_sweeps: int = 10, device="cuda", stream=None) -> dict:
    """Time the plain sweep's candidate shapes for side L and install the fastest
    for L's size class; returns the chosen entry."""
    import torch
    dev = torch.device(device)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    # the lattice, then room for the trials' per-sweep (E, M)
    nbytes = (ising_lattice_bytes(L) + 255) // 256 * 256 + 16 * max(int(trial_sweeps), 2)
    buf = _dev_alloc(nbytes, dev)
    out = ising_tuning()
    check(lib().ising_autotune(int(L), buf.data_ptr(), nbytes, _stream_ptr(st), int(trial_sweeps),
                               ctypes.byref(out)))
    return {k: getattr(out, k) for k in _TUNING_KEYS}


def tuning_get():
    """Installed tuning entries as a list of dicts."""
    n = ctypes.c_int32()
    check(lib().ising_tuning_get(None, 0, ctypes.byref(n)))
    arr = (ising_tuning * max(n.value, 1))()
    check(lib().ising_tuning_get(arr, n.value, ctypes.byref(n)))
    return [{k: getattr(arr[i], k) for k in _TUNING_KEYS} for i in range(n.value)]


def tuning_set(entries):
    arr = (ising_tuning * max(len(entries), 1))()
    for i, e in enumerate(entries):
        for k in _TUNING_KEYS:
            setattr(arr[i], k, e.get(k, 0) if k == "form" else e[k])
    check(lib().ising_tuning_set(arr, len(entries)))


def tuning_clear():
    check(lib().ising_tuning_clear())


def tuning_lookup(L: int) -> dict:
    """The launch shape a lattice of side L created now would use."""
    out = ising_tuning()
    check(lib().ising_tuning_lookup(int(L), ctypes.byref(out)))
    return {k: getattr(out, k) for k in _TUNING_KEYS}


def save_tuning(path: str):
    import json
    with open(path, "w") as f:
        json.dump(tuning_get(), f, indent=1)


def load_tuning(path: str):
    import json
    with open(path) as f:
        tuning_set(json.load(f))


def batch_plan(Ls: Sequence[int], cus: int = 256):
    """(form, grid size, model seconds per sweep) the batched path would use."""
    n = len(Ls)
    arr = (ctypes.c_int64 * max(n, 1))(*[int(L) for L in Ls])
    form, blocks, est = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    check(lib().ising_batch_plan(arr, n, int(cus), ctypes.byref(form), ctypes.byref(blocks),
                                 ctypes.byref(est)))
    return ("packed" if form.value == 1 else "fused"), int(blocks.value), float(est.value)


def multi_sweep(lattices: Sequence[Lattice], n: int, EMs=None, form=None, graph_chunk=-1):
    """n sweeps on every lattice together (same device and stream).
    form: None (cost model), "fused" or "packed"."""
    arr = (ctypes.c_void_p * max(len(lattices), 1))(*[lat.h.value for lat in lattices])
    em_arr = None
    if EMs is not None:
        em_arr = (ctypes.c_void_p * max(len(lattices), 1))(
            *[(e.data_ptr() if e is not None else None) for e in EMs])
    f = {None: -1, "fused": 0, "packed": 1}[form]
    nbytes = ctypes.c_size_t()
    check(lib().ising_multi_sweep_work_bytes(arr, len(lattices), ctypes.byref(nbytes)))
    work = None
    if nbytes.value > 0:
        # the call synchronises the lattices' stream before it returns, so
        # the work buffer may go back to torch's pool right after it
        work = _dev_alloc(nbytes.value, lattices[0].device)
    check(lib().ising_multi_sweep_form(arr, len(lattices), int(n), em_arr, f, int(graph_chunk),
                                       work.data_ptr() if work is not None else None,
                                       int(nbytes.value)))


_BATCH_TUNING_KEYS = ["form", "rpw_max", "wg_per_cu", "graph_chunk", "updates_per_ns",
                      "default_updates_per_ns", "packed_updates_per_ns"]


def multi_autotune(lattices: Sequence[Lattice], trial_sweeps: int = 128) -> dict:
    """Time the batched sweep's fused shapes on copies of these lattices
    (the lattices themselves are not advanced) and install the fastest for
    later batched calls; returns it."""
    arr = (ctypes.c_void_p * max(len(lattices), 1))(*[lat.h.value for lat in lattices])
    nbytes = ctypes.c_size_t()
    check(lib().ising_multi_autotune_bytes(arr, len(lattices), int(trial_sweeps),
                                           ctypes.byref(nbytes)))
    # the call synchronises the lattices' stream before it returns
    buf = _dev_alloc(nbytes.value, lattices[0].device)
    out = ising_batch_tuning()
    check(lib().ising_multi_autotune(arr, len(lattices), int(trial_sweeps), buf.data_ptr(),
                                     int(nbytes.value), ctypes.byref(out)))
    return {k: getattr(out, k) for k in _BATCH_TUNING_KEYS}


def batch_tuning_get() -> dict:
    """The fused shape batched calls use now, and whether it was installed."""
    out = ising_batch_tuning()
    inst = ctypes.c_int32()
    check(lib().ising_batch_tuning_get(ctypes.byref(out), ctypes.byref(inst)))
    d = {k: getattr(out, k) for k in _BATCH_TUNING_KEYS}
    d["installed"] = bool(inst.value)
    return d


def batch_tuning_set(rpw_max: int, wg_per_cu: int, graph_chunk: int):
    t = ising_batch_tuning(0, int(rpw_max), int(wg_per_cu), int(graph_chunk), 0.0, 0.0, 0.0)
    check(lib().ising_batch_tuning_set(ctypes.byref(t)))


def batch_tuning_clear():
    check(lib().ising_batch_tuning_clear())


def reweight(EMs, betas0, discards, task_lattice, task_beta, nblocks: int, stream=None):
    """Per-block reweighted sums of device series (ising_reweight).

    EMs: int64 (n, 2) device tensors; betas0, discards: one per series;
    tasks: task_lattice[k] (series index) reweighted to task_beta[k].
    Returns (sums, shift): float64 device tensors (ntask, nblocks, 5), (ntask,)."""
    import torch
    nl, nt = len(EMs), len(task_lattice)
    dev = EMs[0].device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    for e in EMs:
        if e.dtype != torch.int64 or e.dim() != 2 or e.shape[1] != 2 or not e.is_contiguous():
            raise IsingError(ISING_EINVAL, "reweight: series must be contiguous int64 (n, 2)")
    sums = torch.empty((max(nt, 1), nblocks, 5), dtype=torch.float64, device=dev)
    shift = torch.empty((max(nt, 1),), dtype=torch.float64, device=dev)
    work = _dev_alloc(int(lib().ising_reweight_work_bytes(max(nl, 1), max(nt, 1))), dev)
    # the kernel reads these on stream st after the call returns: tell
    # torch's allocator, so their memory is not reused before st passes it
    for t in (sums, shift, work):
        t.record_stream(st)
    ptrs = (ctypes.c_void_p * max(nl, 1))(*[e.data_ptr() for e in EMs])
    n = (ctypes.c_int64 * max(nl, 1))(*[int(e.shape[0]) for e in EMs])
    d = (ctypes.c_int64 * max(nl, 1))(*[int(v) for v in discards])
    b0 = (ctypes.c_double * max(nl, 1))(*[float(v) for v in betas0])
    tl = (ctypes.c_int32 * max(nt, 1))(*[int(v) for v in task_lattice])
    tb = (ctypes.c_double * max(nt, 1))(*[float(v) for v in task_beta])
    check(lib().ising_reweight(nl, ptrs, n, d, b0, nt, tl, tb, int(nblocks), sums.data_ptr(),
                               shift.data_ptr(), work.data_ptr(), int(work.numel()),
                               _stream_ptr(st)))
    return sums, shift


def fss_moments(sums, sites):
    """(est, err, u4_rep) from host per-block sums (ntask, B, 5) (ising_fss_moments):
    est/err (ntask, 3) = (U4, <E>/N, <|M|>/N) and jackknife errors, u4_rep (ntask, B)."""
    import numpy as np
    S = np.ascontiguousarray(np.asarray(sums, dtype=np.float64))
    nt, B = S.shape[0], S.shape[1]
    N = np.ascontiguousarray(np.asarray(sites, dtype=np.int64).reshape(nt))
    est = np.empty((nt, 3))
    err = np.empty((nt, 3))
    rep = np.empty((nt, B))
    check(lib().ising_fss_moments(S.ctypes.data, nt, B,
                                  N.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  est.ctypes.data, err.ctypes.data, rep.ctypes.data))
    return est, err, rep


def autocorr_time(x, c: float = 5.0):
    """(tau, window) of a host series (ising_autocorr_time); window -1 when the
    series is too short for its correlations."""
    a = np.ascontiguousarray(x, dtype=np.float64)
    tau, W = ctypes.c_double(), ctypes.c_int64()
    check(lib().ising_autocorr_time(a.ctypes.data, int(a.size), float(c), ctypes.byref(tau),
                                    ctypes.byref(W)))
    return float(tau.value), int(W.value)


def binder_crossing(T, Ua, Ub, Ua_rep=None, Ub_rep=None):
    """(T*, U*, err T*, err U*) of two U4 curves (ising_binder_crossing)."""
    import numpy as np
    T = np.ascontiguousarray(T, dtype=np.float64)
    a = np.ascontiguousarray(Ua, dtype=np.float64)
    b = np.ascontiguousarray(Ub, dtype=np.float64)
    out = np.empty(4)
    ra = rb = None
    B = 0
    if Ua_rep is not None:
        ra = np.ascontiguousarray(Ua_rep, dtype=np.float64)
        rb = np.ascontiguousarray(Ub_rep, dtype=np.float64)
        B = ra.shape[0]
    check(lib().ising_binder_crossing(T.ctypes.data, len(T), a.ctypes.data, b.ctypes.data,
                                      None if ra is None else ra.ctypes.data,
                                      None if rb is None else rb.ctypes.data, B,
                                      out.ctypes.data))
    return tuple(float(v) for v in out)


def binder_curves(EMs, Ls, temps, discard: int, T_grid, nblocks: int = 20, stream=None):
    """U4 curves on T_grid for every lattice size among Ls: each grid point is
    reweighted from the run of that size whose temperature is nearest.
    Returns {L: (est (K, 3), err (K, 3), u4_rep (nblocks, K))}."""
    import numpy as np
    Ls = [int(v) for v in Ls]
    temps = np.asarray(temps, dtype=np.float64)
    T_grid = np.asarray(T_grid, dtype=np.float64)
    sizes = sorted(set(Ls))
    tl, tb, tsite = [], [], []
    for L in sizes:
        runs = [i for i, v in enumerate(Ls) if v == L]
        for T in T_grid:
            i = runs[int(np.argmin(np.abs(temps[runs] - T)))]
            tl.append(i)
            tb.append(1.0 / T)
            tsite.append(L * L)
    sums, _ = reweight(EMs, [1.0 / t for t in temps], [discard] * len(EMs), tl, tb, nblocks,
                       stream)
    est, err, rep = fss_moments(sums.cpu().numpy(), tsite)
    K = len(T_grid)
    return {L: (est[j * K:(j + 1) * K], err[j * K:(j + 1) * K], rep[j * K:(j + 1) * K].T.copy())
            for j, L in enumerate(sizes)}


def series_moments(series, discard: int = 0):
    """(sum_M2, sum_M4, n_kept) of an (n, 2) int64 (E, M) series over sweeps
    discard .. n - 1: exact integer sums, each rounded once to double
    (ising_series_moments; host only)."""
    import numpy as np
    a = np.ascontiguousarray(np.asarray(series, dtype=np.int64).reshape(-1, 2))
    m2, m4, kept = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    check(lib().ising_series_moments(a.ctypes.data if a.size else None, a.shape[0], int(discard),
                                     ctypes.byref(m2), ctypes.byref(m4), ctypes.byref(kept)))
    return m2.value, m4.value, kept.value


class Server:
    """Continuous-batching server over a device arena (a torch uint8 tensor)."""

    def __init__(self, arena_bytes: int, quantum_sweeps: int = 100, device="cuda", stream=None):
        import torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.arena = _dev_alloc(arena_bytes, self.device)
        s = ctypes.c_void_p()
        check(lib().ising_server_create(self.arena.data_ptr(), int(arena_bytes),
                                        _stream_ptr(self.stream), int(quantum_sweeps),
                                        ctypes.byref(s)))
        self.s = s
        self._buffers = {}

    def close(self):
        if getattr(self, "s", None):
            lib().ising_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, requests):
        """requests: iterable of dicts with L, beta, seed, stream_id, init, n_sweeps and
        optional n_discard, record_series, return_spins.  Returns the tickets."""
        requests = list(requests)
        arr = (ising_request * max(len(requests), 1))()
        keep = []
        for i, r in enumerate(requests):
            q = arr[i]
            q.L, q.beta, q.seed = int(r["L"]), float(r["beta"]), int(r.get("seed", 1))
            q.stream_id, q.init = int(r.get("stream_id", 0)), int(r.get("init", INIT_HOT))
            q.n_sweeps, q.n_discard = int(r["n_sweeps"]), int(r.get("n_discard", 0))
            flags = 0
            series = spins = None
            if r.get("record_series"):
                flags |= REQ_RECORD_SERIES
                series = np.zeros((q.n_sweeps, 2), dtype=np.int64)
                q.EM_series = series.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            if r.get("return_spins"):
                flags |= REQ_RETURN_SPINS
                spins = np.zeros((q.L, q.L), dtype=np.int8)
                q.spins_out = spins.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
            q.flags = flags
            keep.append((series, spins))
        tickets = (ctypes.c_uint64 * max(len(requests), 1))()
        check(lib().ising_batch_submit(self.s, arr, len(requests), tickets))
        out = [int(tickets[i]) for i in range(len(requests))]
        for t, k in zip(out, keep):
            self._buffers[t] = k
        return out

    def step(self) -> bool:
        """One quantum; True while work remains."""
        return check(lib().ising_server_step(self.s), ok=(ISING_OK, ISING_AGAIN)) == ISING_AGAIN

    def poll(self, ticket: int):
        """None while running; else a dict with the result (and series/spins if requested)."""
        r = ising_result()
        code = check(lib().ising_poll(self.s, int(ticket), ctypes.byref(r)),
                     ok=(ISING_OK, ISING_AGAIN))
        if code == ISING_AGAIN:
            return None
        series, spins = self._buffers.pop(int(ticket), (None, None))
        return {"ticket": int(r.ticket), "E_final": int(r.E_final), "M_final": int(r.M_final),
                "sweeps_done": int(r.sweeps_done), "sum_M2": float(r.sum_M2),
                "sum_M4": float(r.sum_M4), "n_kept": int(r.n_kept), "t_arrive": r.t_arrive,
                "t_admit": r.t_admit, "t_done": r.t_done, "series": series, "spins": spins}

    def inject_fault(self, quantum_index: int):
        check(lib().ising_server_inject_fault(self.s, int(quantum_index)))

    def stats(self):
        out = (ctypes.c_int64 * 6)()
        check(lib().ising_server_stats(self.s, out))
        keys = ["quanta", "admitted", "done", "bytes_in_use", "peak_bytes", "faults_recovered"]
        return dict(zip(keys, [int(v) for v in out]))

    def run_until_idle(self, max_steps: int = 10 ** 9):
        for _ in range(max_steps):
            if not self.step():
                return
        raise RuntimeError("server did not become idle")
