"""The C ABI library loads on the CPU and exports every declared symbol;
argument validation that happens before any device work (CPU only)."""
import ctypes
import math
import re
import subprocess
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ising.h")).read()
    return sorted(set(re.findall(r"ISING_API[^;(]*?\b(ising_\w+)\s*\(", text, flags=re.S)))


@pytest.fixture(scope="module")
def L():
    from paper_1007_3726_amd import ising
    return ising.lib()


def test_header_declares_the_entry_points():
    names = _declared()
    for required in ["ising_create", "ising_set_beta", "ising_sweep", "ising_measure",
                     "ising_batch_submit", "ising_poll", "ising_multi_sweep"]:
        assert required in names


def test_every_declared_symbol_is_exported(L):
    path = os.path.join(ROOT, "paper_1007_3726_amd", "libising.so")
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (ising_\w+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        assert hasattr(L, n)


def test_lattice_bytes(L):
    from paper_1007_3726_amd import ising
    scratch = 256 + 2 * 2048 * 16

    def planes(L):
        b = 2 * L * (((L // 2) + 63) // 64) * 8
        return (b + 255) // 256 * 256

    assert ising.ising_lattice_bytes(64) == planes(64) + scratch
    assert ising.ising_lattice_bytes(16384) == 2 * 16384 * 128 * 8 + scratch
    assert ising.ising_lattice_bytes(262144) == 2 * 262144 * 2048 * 8 + scratch
    assert ising.ising_lattice_bytes(130) == planes(130) + scratch
    for bad in (-2, 0, 2, 3, 5, 63, 2 ** 21 + 2):
        assert ising.ising_lattice_bytes(bad) == 0


def test_create_validation_before_device_work(L):
    h = ctypes.c_void_p()
    buf = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    assert L.ising_create(5, 1, 0, 0, buf, 1 << 20, None, ctypes.byref(h)) == -1
    assert L.ising_create(64, 1, 0, 3, buf, 1 << 20, None, ctypes.byref(h)) == -1
    assert L.ising_create(64, 1, 1 << 30, 0, buf, 1 << 20, None, ctypes.byref(h)) == -1
    assert L.ising_create(64, 1, 0, 0, None, 1 << 20, None, ctypes.byref(h)) == -1
    assert L.ising_create(64, 1, 0, 0, ctypes.c_void_p(4097), 1 << 20, None, ctypes.byref(h)) == -1
    assert L.ising_create(64, 1, 0, 0, buf, 100, None, ctypes.byref(h)) == -2
    assert b"dev_bytes" in L.ising_last_error()
    assert L.ising_create(64, 1, 0, 0, buf, 1 << 20, None, None) == -1


def test_null_handles_are_rejected(L):
    assert L.ising_set_beta(None, 1.0) == -1
    assert L.ising_sweep(None, 1, None) == -1
    assert L.ising_destroy(None) == 0
    E = ctypes.c_int64()
    assert L.ising_measure(None, ctypes.byref(E), ctypes.byref(E)) == -1


def test_tuning_table_roundtrip(L):
    from paper_1007_3726_amd import ising
    ising.tuning_clear()
    e = {"L_min": 8192, "L_max": 16383, "form": ising.ISING_FORM_TILE, "rpw": 2,
         "max_blocks": 1024, "small_lds_bytes": 0, "updates_per_ns": 1.5}
    ising.tuning_set([e])
    assert ising.tuning_get() == [e]
    e2 = dict(e, rpw=4)
    ising.tuning_set([e2])  # same class replaces
    assert ising.tuning_get() == [e2]
    e3 = dict(e, form=ising.ISING_FORM_STRIP, rpw=1024)  # strips allow long tasks
    ising.tuning_set([e3])
    assert ising.tuning_get() == [e3]
    for bad in (dict(e, max_blocks=4096), dict(e, rpw=-1), dict(e, L_max=10),
                dict(e, small_lds_bytes=1 << 20), dict(e, rpw=32), dict(e, form=2),
                dict(e3, rpw=(1 << 21) + 1)):
        with pytest.raises(ising.IsingError):
            ising.tuning_set([bad])
    ising.tuning_clear()
    assert ising.tuning_get() == []
    # built-in defaults: LDS-resident up to 128^2, tiles above
    assert ising.tuning_lookup(64)["small_lds_bytes"] >= 2 * 64 * 8
    assert ising.tuning_lookup(4096)["form"] == ising.ISING_FORM_TILE
    assert ising.tuning_lookup(16384)["form"] == ising.ISING_FORM_TILE
    # the size rule resolved: as many row groups per wave (4, 2) as keep
    # >= 2048 tiles of 4 x R x rpw rows x 64-word segments
    assert ising.tuning_lookup(16384)["rpw"] == 4    # 1024 x 2 tiles of 16 rows
    assert ising.tuning_lookup(262144)["rpw"] == 4
    assert ising.tuning_lookup(8192)["rpw"] == 1     # 1024 tiles at rpw 2: too few
    assert ising.tuning_lookup(1024)["rpw"] == 1     # too few tiles for 2
    ising.tuning_set([e2])
    assert ising.tuning_lookup(9000)["rpw"] == 4 and ising.tuning_lookup(9000)["L_min"] == 8192
    ising.tuning_clear()


def test_missing_library_fails_loudly():
    """Without libising.so the binding raises: there is no CPU fallback."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1007_3726_amd import ising\n"
            "ising.LIB_PATH = '/nonexistent/libising.so'\n"
            "try:\n"
            "    ising.Lattice(64, beta=0.4, device='cpu')\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert "raised:" in r.stdout and "no fallback" in r.stdout, r.stdout + r.stderr


def test_rng_state_sizes(L):
    from paper_1007_3726_amd import ising
    for m in (10, 16, 22, 28):
        assert ising.ising_pool_bytes(m) == 16 << m
    for bad in (-1, 0, 9, 29, 64):
        assert ising.ising_pool_bytes(bad) == 0
    # one uint32 state per 64-site word of each colour plane
    assert ising.ising_lcg_bytes(4) == 2 * 4 * 1 * 4
    assert ising.ising_lcg_bytes(16384) == 2 * 16384 * 128 * 4
    assert ising.ising_lcg_bytes(130) == 2 * 130 * 2 * 4
    for bad in (-2, 0, 2, 5, 2 ** 21 + 2):
        assert ising.ising_lcg_bytes(bad) == 0
    assert L.ising_set_rng(None, 0, None, 0) == -1


def test_strip_validation_before_device_work(L):
    part = 2 * 2048 * 8
    assert L.ising_strip_bytes(128, 1) == 2 * 3 * 1 * 8 + part
    assert L.ising_strip_bytes(262144, 32768) == 2 * 32770 * 2048 * 8 + part
    for Lb, rows in ((130, 1), (64, 1), (128, 0), (128, 129), (2 ** 21, 2 ** 21), (2 ** 22, 1)):
        assert L.ising_strip_bytes(Lb, rows) == 0, (Lb, rows)
    h = ctypes.c_void_p()
    buf = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    need = L.ising_strip_bytes(256, 64)
    args = dict(L=256, y0=0, rows=64, seed=1, sid=0, init=2, buf=buf, nbytes=need)

    def create(**kw):
        a = dict(args, **kw)
        return L.ising_strip_create(a["L"], a["y0"], a["rows"], a["seed"], a["sid"], a["init"],
                                    a["buf"], a["nbytes"], None, ctypes.byref(h))

    assert create(L=130) == -1
    assert create(rows=0) == -1
    assert create(y0=200) == -1  # rows 200 .. 263 pass the lattice's end
    assert create(y0=-1) == -1
    assert create(init=3) == -1
    assert create(sid=1 << 30) == -1
    assert create(nbytes=need - 1) == -2
    assert create(buf=None) == -2
    assert create(buf=ctypes.c_void_p(4100)) == -1  # not 8-byte aligned
    assert L.ising_strip_create(256, 0, 64, 1, 0, 2, buf, need, None, None) == -1
    assert L.ising_strip_set_beta(None, 1.0) == -1
    assert L.ising_strip_step(None, 0, 0, None) == -1
    assert L.ising_strip_exchange(None, 1, 0) == -1
    assert L.ising_strip_get_rows(None, None) == -1
    assert L.ising_strip_destroy(None) == 0
    ptr, nb = ctypes.c_void_p(), ctypes.c_size_t()
    assert L.ising_strip_row(None, 0, 0, ctypes.byref(ptr), ctypes.byref(nb)) == -1
    assert L.ising_strip_combine(None, 1, 1, 256, None, None) == -1
    assert L.ising_strip_combine(ctypes.c_void_p(4096), 1, 0, 256, ctypes.c_void_p(4096),
                                 None) == 0  # nothing to combine: no device work


def test_server_validation_before_device_work(L):
    s = ctypes.c_void_p()
    arena = ctypes.c_void_p(1 << 20)  # never dereferenced
    assert L.ising_server_create(arena, 1 << 20, None, 4, None) == -1
    assert L.ising_server_create(None, 1 << 20, None, 4, ctypes.byref(s)) == -1
    assert L.ising_server_create(ctypes.c_void_p((1 << 20) + 8), 1 << 20, None, 4,
                                 ctypes.byref(s)) == -1  # not 256-byte aligned
    assert L.ising_server_create(arena, 1 << 20, None, 0, ctypes.byref(s)) == -1
    # the table region takes at least 4 KiB and at most half of the arena
    assert L.ising_server_create(arena, 4096, None, 4, ctypes.byref(s)) == -1
    assert L.ising_server_step(None) == -1
    assert L.ising_batch_submit(None, None, 0, None) == -1
    assert L.ising_poll(None, 1, None) == -1
    assert L.ising_server_inject_fault(None, 0) == -1
    assert L.ising_server_destroy(None) == 0


def test_batch_and_reweight_validation_before_device_work(L):
    assert L.ising_multi_sweep(None, 1, 1, None, None, 0) == -1
    two = (ctypes.c_void_p * 2)(None, None)
    assert L.ising_multi_sweep(two, 2, 1, None, None, 0) == -1  # NULL handles
    assert L.ising_multi_sweep(two, -1, 1, None, None, 0) == -1
    assert L.ising_multi_sweep_form(None, 1, 1, None, 0, -1, None, 0) == -1
    nb = ctypes.c_size_t(7)
    assert L.ising_multi_sweep_work_bytes(two, 2, ctypes.byref(nb)) == -1 and nb.value == 0
    assert L.ising_multi_sweep_work_bytes(two, 0, None) == -1
    i64 = ctypes.c_int64
    f64 = ctypes.c_double
    em = (ctypes.c_void_p * 1)(4096)  # never dereferenced
    nsw, disc, b0 = (i64 * 1)(100), (i64 * 1)(20), (f64 * 1)(0.44)
    tl, tb = (ctypes.c_int32 * 1)(0), (f64 * 1)(0.45)
    sums = ctypes.c_void_p(8192)
    work = ctypes.c_void_p(1 << 16)  # 256-byte aligned, never dereferenced
    need = int(L.ising_reweight_work_bytes(1, 1))
    assert need >= 256 + 16 and L.ising_reweight_work_bytes(0, 1) == 0
    assert L.ising_reweight_work_bytes(3, 1000) >= 1000 * 16

    def rw(nlat=1, em=em, nsw=nsw, disc=disc, b0=b0, ntask=1, tl=tl, tb=tb, nblocks=20,
           sums=sums, work=work, nwork=need):
        return L.ising_reweight(nlat, em, nsw, disc, b0, ntask, tl, tb, nblocks, sums, None,
                                work, nwork, None)

    assert rw(work=None) == -2
    assert rw(work=ctypes.c_void_p((1 << 16) + 8)) == -2  # misaligned
    assert rw(nwork=need - 1) == -2

    assert rw(nlat=0) == -1
    assert rw(ntask=0) == -1
    assert rw(em=None) == -1
    assert rw(sums=None) == -1
    assert rw(nblocks=0) == -1
    assert rw(nblocks=1 << 20) == -1
    assert rw(disc=(i64 * 1)(-1)) == -1
    assert rw(disc=(i64 * 1)(90)) == -1  # 10 kept sweeps < 20 blocks
    assert rw(b0=(f64 * 1)(float("nan"))) == -1
    assert rw(b0=(f64 * 1)(-0.1)) == -1
    assert rw(tl=(ctypes.c_int32 * 1)(1)) == -1  # no series 1
    assert rw(tb=(f64 * 1)(float("inf"))) == -1
