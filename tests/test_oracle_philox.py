"""Pins of the oracle's Philox4x32-10 and samplers.

The generator is pinned to an independent implementation of the same published
definition (rocRAND's host-callable Philox4x32-10 engine, compiled here from its
header), in the oracle's exact counter layout.  The samplers are pinned by exactness
and distribution tests.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_kat(tmp_path_factory):
    cxx = shutil.which("g++")
    inc = "/opt/rocm/include"
    if cxx is None or not os.path.exists(os.path.join(inc, "rocrand", "rocrand_philox4x32_10.h")):
        pytest.skip("g++ or rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("kat") / "kat")
    subprocess.run([cxx, "-O1", "-D__HIP_PLATFORM_AMD__", "-I" + inc,
                    os.path.join(HERE, "rocrand_philox_kat.cpp"), "-o", exe], check=True)

    def run(rows):
        text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)

    return run


def test_philox_matches_rocrand(rocrand_kat):
    rng = np.random.default_rng(123)
    n = 3000
    seeds = rng.integers(0, 2 ** 63, n, dtype=np.uint64)
    seeds[:5] = [0, 1, 2 ** 32 - 1, 2 ** 32, 2 ** 63 - 1]
    c0 = rng.integers(0, 2 ** 32, n, dtype=np.uint64)
    c1 = rng.integers(0, 2 ** 30, n, dtype=np.uint64)
    c2 = rng.integers(0, 2 ** 32, n, dtype=np.uint64)
    c3 = rng.integers(0, 2 ** 32, n, dtype=np.uint64)
    c0[:3] = 0
    c1[:3] = 0
    c2[:3] = 0
    c3[:3] = 0
    rows = np.stack([seeds, c0, c1, c2, c3], axis=1)
    ref = rocrand_kat(rows)
    for i in range(n):
        k0, k1 = philox.key_of(int(seeds[i]))
        got = philox.philox4x32_10(c0[i], c1[i], c2[i], c3[i], k0, k1)
        assert [int(g) for g in got] == [int(r) for r in ref[i]], i


def test_draw_layout_matches_rocrand(rocrand_kat):
    """draw(ids, step, species, stream, seed) uses counter (id, 0, step, (species << 8) | stream)."""
    ids = np.array([0, 1, 7, 123456, 2 ** 32 - 1], dtype=np.uint64)
    for seed, step, s, stream in [(0, 0, 0, 0), (5, 17, 1, 2), (2 ** 40 + 3, 2 ** 31, 1, 0xFF)]:
        got = np.stack(philox.draw(ids, step, s, stream, seed), axis=1)
        rows = [[seed, int(i), 0, step, (s << 8) | stream] for i in ids]
        assert np.array_equal(got, rocrand_kat(rows))


def test_uniform_exact_and_open_interval():
    w = np.array([0, 511, 512, 2 ** 32 - 1, 0x80000000], dtype=np.uint64)
    u = philox.uniform(w)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24
    assert u[2] == 3 * 2.0 ** -24
    assert u[3] == 1.0 - 2.0 ** -24
    assert np.all(u.astype(np.float32).astype(np.float64) == u)  # exactly representable in FP32
    assert np.all((u > 0) & (u < 1))


def test_uniformity_and_independence():
    ids = np.arange(200_000, dtype=np.uint64)
    w = philox.draw(ids, 9, 0, 0, 42)
    for k in range(4):
        u = philox.uniform(w[k])
        assert stats.kstest(u, "uniform").pvalue > 1e-4
    # words of one call are uncorrelated
    u0, u1 = philox.uniform(w[0]), philox.uniform(w[1])
    assert abs(np.corrcoef(u0, u1)[0, 1]) < 0.02
    # neighbouring counters are uncorrelated
    assert abs(np.corrcoef(u0[:-1], u0[1:])[0, 1]) < 0.02


def test_normals_and_directions():
    ids = np.arange(200_000, dtype=np.uint64)
    w = philox.draw(ids, 3, 1, 1, 7)
    z0, z1 = philox.normal_pair(w[0], w[1])
    for z in (z0, z1):
        assert stats.kstest(z, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 0.02
    n = philox.direction(w[2], w[3])
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-12)
    # isotropy: cos(chi) uniform on [-1, 1], azimuth uniform on [0, 2 pi)
    assert stats.kstest((n[:, 0] + 1) / 2, "uniform").pvalue > 1e-4
    az = np.mod(np.arctan2(n[:, 2], n[:, 1]), 2 * np.pi) / (2 * np.pi)
    assert stats.kstest(az, "uniform").pvalue > 1e-4
