"""The allocation-free warm-start loader (pic_load_profiles_noalloc) against the loader that
allocates its staging (pic_load_profiles), through the C ABI: two calls in a row, the second
with fewer profile points and lower densities, each compared per id (the same kernels draw
the same particles, so the states must be bitwise equal), with the field solved after the
load; and the size limit is rejected with PIC_EINVAL."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from gpu_common import log
from paper_1608_04601_amd import binding as B

pytestmark = pytest.mark.gpu


def _profiles(npts, peak, gap):
    z = np.linspace(0.0, gap, npts)
    s = np.sin(np.pi * z / gap)
    return dict(n_e=peak * s ** 2 + 1e12, n_i=peak * s + 1e12, mean_energy_e=2.0 + 3.0 * s,
                flux_i=4e18 * np.cos(np.pi * z / gap))


def _state(d):
    out = []
    for sp in (0, 1):
        p = d.particles(sp)
        k = np.argsort(p["id"])
        out.append({key: v[k] for key, v in p.items()})
    return out, d.counters(), d.fields()


def _same(a, b, tag):
    (pa, ca, fa), (pb, cb, fb) = a, b
    for sp in (0, 1):
        for key in ("id", "x", "vx", "vy", "vz"):
            assert np.array_equal(pa[sp][key], pb[sp][key]), (tag, sp, key)
    assert ca["n_alive"] == cb["n_alive"] and ca["next_id"] == cb["next_id"], tag
    for key in ("E", "phi", "Q"):
        assert np.array_equal(fa[key], fb[key]), (tag, key)


def test_noalloc_loader_equals_allocating_loader_twice():
    disc = W.small_argon(seed=4, n_super=20_000).replace(capacity=(200_000, 200_000))
    for call, (npts, peak) in enumerate(((129, 4e15), (33, 1.5e15))):
        prof = _profiles(npts, peak, disc.gap_m)
        log(f"no-alloc loader call {call}: {npts} points, peak {peak:.1e}")
        with B.Discharge(disc) as ref, B.Discharge(disc) as got:
            B.pic_load_profiles(ref.h, prof["n_e"], prof["n_i"], prof["mean_energy_e"], prof["flux_i"])
            B.pic_load_profiles_noalloc(got.h, prof["n_e"], prof["n_i"], prof["mean_energy_e"], prof["flux_i"])
            a, b = _state(ref), _state(got)
            assert a[1]["n_alive"][0] > 1000
            _same(a, b, call)
            ref.step(5)
            got.step(5)
            _same(_state(ref), _state(got), (call, "stepped"))


def test_noalloc_loader_rejects_too_many_points():
    disc = W.small_argon(seed=4, n_super=2_000)
    prof = _profiles(1025, 1e15, disc.gap_m)
    with B.Discharge(disc) as d:
        arrs = [np.ascontiguousarray(prof[k]) for k in ("n_e", "n_i", "mean_energy_e", "flux_i")]
        ptrs = [a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs]
        rc = B.load_library().pic_load_profiles_noalloc(d.h, 1025, *ptrs)
        assert rc == B.PIC_EINVAL
        assert b"PIC_NOALLOC_MAX_POINTS" in B.load_library().pic_last_error(d.h)
