"""Pins the oracle's Philox4x32-10 and its keying to independent implementations.

The oracle's generator is checked against two header implementations that
are executed, not copied: ATen's at::philox_engine
(torch/include/ATen/core/PhiloxRNGEngine.h) and rocRAND's
philox4x32_10_engine::ten_rounds (rocrand/rocrand_philox4x32_10.h).
A dropped round, a wrong multiplier, a swapped output word or a wrong key
bump makes every comparison fail.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _build(src, compiler, extra):
    out = os.path.join(tempfile.gettempdir(), "ising_xref_" + os.path.basename(src) + ".bin")
    if not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        subprocess.run([compiler, "-O1", "-std=c++17", *extra, "-o", out, src], check=True,
                       stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return out


@pytest.fixture(scope="module")
def torch_engine():
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    return _build(os.path.join(HERE, "xref", "torch_philox.cpp"), "g++", ["-I" + inc])


@pytest.fixture(scope="module")
def rocrand_engine():
    if not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers not present")
    return _build(os.path.join(HERE, "xref", "rocrand_philox.cpp"), "hipcc", [])


def _run(binary, lines):
    r = subprocess.run([binary], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       check=True)
    return [[int(v) for v in ln.split()] for ln in r.stdout.strip().splitlines()]


def test_philox_block_matches_rocrand(rocrand_engine):
    rng = np.random.default_rng(11)
    cases = [[0] * 6, [0xFFFFFFFF] * 6]
    cases += [[int(v) for v in rng.integers(0, 2 ** 32, 6)] for _ in range(300)]
    ref = _run(rocrand_engine, [" ".join(map(str, c)) for c in cases])
    for c, r in zip(cases, ref):
        assert oracle.philox4x32_10(c[:4], c[4:]) == r, c


def test_philox_block_matches_aten(torch_engine):
    # at::philox_engine(seed, subsequence, offset): key = (lo, hi)(seed),
    # counter = (lo, hi)(offset), (lo, hi)(subsequence).
    rng = np.random.default_rng(12)
    cases = [(0, 0, 0), (2 ** 64 - 1, 2 ** 64 - 1, 2 ** 64 - 1)]
    cases += [tuple(int(v) for v in rng.integers(0, 2 ** 63, 3)) for _ in range(300)]
    ref = _run(torch_engine, ["%d %d %d" % c for c in cases])
    for (seed, sub, off), r in zip(cases, ref):
        ctr = [off & 0xFFFFFFFF, off >> 32, sub & 0xFFFFFFFF, sub >> 32]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        assert oracle.philox4x32_10(ctr, key) == r


def test_site_keying_matches_aten(torch_engine):
    # uniform(seed, sid, phase, t, L, x, y) is output j of the block with
    # offset g and subsequence t | ((sid << 2 | phase) << 32), where
    # i = y*(L/2) + x//2, g = i // 4, j = i % 4.
    rng = np.random.default_rng(13)
    cases, lines = [], []
    for _ in range(400):
        L = int(rng.choice([4, 6, 10, 64, 130, 16384, 262144]))
        x, y = int(rng.integers(0, L)), int(rng.integers(0, L))
        seed = int(rng.integers(0, 2 ** 63))
        sid = int(rng.integers(0, 2 ** 30))
        phase = int(rng.integers(0, 4))
        t = int(rng.integers(0, 2 ** 32))
        i = y * (L // 2) + x // 2
        sub = t | (((sid << 2) | phase) << 32)
        cases.append((seed, sid, phase, t, L, x, y, i % 4))
        lines.append("%d %d %d" % (seed, sub, i // 4))
    ref = _run(torch_engine, lines)
    for (seed, sid, phase, t, L, x, y, j), r in zip(cases, ref):
        assert oracle.uniform(seed, sid, phase, t, L, x, y) == r[j]


def test_uniform_is_uniform():
    # coarse chi-square on the top 4 bits of 2^14 distinct site uniforms
    L = 512
    vals = np.array([oracle.uniform(5, 0, 0, 3, L, x, y) for y in range(64) for x in range(0, L, 2)],
                    dtype=np.uint64)
    counts = np.bincount((vals >> 28).astype(np.int64), minlength=16)
    exp = len(vals) / 16
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 50.0  # 15 dof, p ~ 1e-5
