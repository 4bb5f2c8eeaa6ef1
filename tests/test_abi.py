"""C-ABI contract checks that need no GPU: the library loads, exports every function that
include/pic1d.h declares, the ctypes layouts match the C layouts, and invalid
configurations are rejected on the host with PIC_EINVAL before any device work."""
import ctypes as C
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W
from paper_1608_04601_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic1d.h")
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions():
    names = set()
    for path in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        names |= set(re.findall(r"\b((?:pic|mlp)_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_function():
    lib = B.load_library()
    names = declared_functions()
    assert set(names) == set(B.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T ((?:pic|mlp)_[a-z_]+)$", out, flags=re.M))
    for n in names:
        assert n in exported, n
        assert getattr(lib, n) is not None


STRUCTS = {
    "pic_xsec": B.pic_xsec, "pic_config": B.pic_config, "pic_moments_out": B.pic_moments_out,
    "pic_counters": B.pic_counters, "pic_derived": B.pic_derived, "pic_tuning": B.pic_tuning, "pic_diag_out": B.pic_diag_out,
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_struct_layouts_match_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pic1d.h"', 'int main(void) {']
    for name, cls in STRUCTS.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for name, cls in STRUCTS.items():
        assert got[(name, "size")] == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)


def _bad(**kw):
    return W.small_argon(n_super=1000).replace(**kw)


@pytest.mark.parametrize("disc, msg", [
    (_bad(gap_m=0.0), "gap_m"),
    (_bad(pressure_Pa=-1.0), "pressure"),
    (_bad(dt_s=float("nan")), "dt_s"),
    (_bad(n_cells=1), "n_cells"),
    (_bad(n_cells=4097), "n_cells"),
    (_bad(capacity=(10, 10)), "n_init_super"),
    (_bad(n_super=(0, 10)), "n_init_super"),
    (_bad(moments_every=0), "moments_every"),
    (_bad(sort_every=-1), "sort_every"),
    (_bad(max_births_per_step=0), "max_births"),
    (_bad(processes=tuple([W.argon_like()[0]] * 17)), "n_xsec"),
    (_bad(processes=(W.Process(W.E_ELASTIC, 0, 0.0, 0.1, 0.0, np.array([1e-19])),)), "n_points"),
    (_bad(processes=(W.Process(W.E_ELASTIC, 0, 0.0, 0.1, 0.0, np.array([1e-19, -1.0])),)), "sigma"),
    (_bad(processes=(W.Process(W.E_ELASTIC, 0, 0.0, 0.0, 0.0, np.array([1e-19, 1e-19])),)), "energies"),
    (_bad(processes=(W.Process(7, 0, 0.0, 0.1, 0.0, np.array([1e-19, 1e-19])),)), "kind"),
    (_bad(processes=(W.Process(0, 2, 0.0, 0.1, 0.0, np.array([1e-19, 1e-19])),)), "frame"),
])
def test_invalid_config_rejected_on_host(disc, msg):
    with pytest.raises(B.PicError) as e:
        B.pic_init(B.Config(disc))
    assert e.value.status == B.PIC_EINVAL
    assert msg in str(e.value)
    assert msg in B.pic_last_error(None)


def test_null_arguments():
    lib = B.load_library()
    lib.pic_free(None)  # NULL-safe
    assert lib.pic_step(None, 1) == B.PIC_EINVAL
    assert lib.pic_sync(None) == B.PIC_EINVAL
    assert lib.pic_init(None, None, None) == B.PIC_EINVAL
    h = C.c_void_p()
    assert lib.pic_init(None, None, C.byref(h)) == B.PIC_EINVAL and not h


def test_batch_null_and_invalid_arguments():
    lib = B.load_library()
    lib.pic_batch_free(None)  # NULL-safe
    assert lib.pic_batch_step(None, 1) == B.PIC_EINVAL
    assert lib.pic_batch_sync(None) == B.PIC_EINVAL
    b = C.c_void_p()
    assert lib.pic_batch_init(None, 1, None, C.byref(b)) == B.PIC_EINVAL and not b
    cfg = B.Config(W.small_argon(n_super=100))
    assert lib.pic_batch_init(C.byref(cfg.c), 0, None, C.byref(b)) == B.PIC_EINVAL and not b
    assert b"n must be" in lib.pic_batch_last_error(None)
    bad = B.Config(_bad(n_cells=1))
    arr = (B.pic_config * 2)(cfg.c, bad.c)
    assert lib.pic_batch_init(arr, 2, None, C.byref(b)) == B.PIC_EINVAL and not b
    assert b"discharge 1" in lib.pic_batch_last_error(None)


def test_mlp_invalid_arguments_rejected_on_host():
    L = B.load_library()
    h = C.c_void_p()
    for args in ((0, 8, 1, 4, 16), (4, 8, 17, 4, 16), (4, 8, 1, 4, 0), (4, 5000, 1, 4, 16)):
        assert L.mlp_init(*args, 0, None, C.byref(h)) == B.PIC_EINVAL
        assert h.value is None
        assert L.mlp_last_error(None)
    assert L.mlp_init(4, 8, 1, 4, 16, 0, None, None) == B.PIC_EINVAL
    assert L.mlp_train_step(None, None, None, 1, 1e-3, None) == B.PIC_EINVAL
    L.mlp_free(None)


def test_new_entry_points_reject_null_on_host():
    """Batches, warm start, diagnostics and current drive: NULL handles are rejected before
    any device work, and a negative current target is an invalid configuration."""
    L = B.load_library()
    for f, args in ((L.pic_batch_set_graph, (None, 10)), (L.pic_set_graph, (None, 10)),
                    (L.pic_batch_autotune, (None, 10, None)),
                    (L.pic_batch_rebalance, (None,)), (L.pic_batch_timing, (None, 1, None, None)),
                    (L.pic_batch_set_record_decisions, (None, 1)),
                    (L.pic_diag_config, (None, 10, 20.0)), (L.pic_diag_sample, (None,)),
                    (L.pic_diag_read, (None, None, 0)), (L.pic_electrode_fluxes, (None, 10, None, None)),
                    (L.pic_load_profiles, (None, 3, None, None, None, None))):
        assert f(*args) == B.PIC_EINVAL, f.__name__
    n = C.c_int64()
    assert L.pic_batch_graph_launches(None, C.byref(n)) == B.PIC_EINVAL
    assert L.pic_graph_launches(None, C.byref(n)) == B.PIC_EINVAL
    assert L.pic_launch_shape(None, None, None, None) == B.PIC_EINVAL
    assert L.mlp_num_params(None, C.byref(n)) == B.PIC_EINVAL


@pytest.mark.parametrize("j0", [-1.0, float("nan"), float("inf")])
def test_invalid_current_target_rejected_on_host(j0):
    cfg = B.Config(W.small_argon(n_super=100).replace(j0_target_A_m2=j0))
    h = C.c_void_p()
    assert B.load_library().pic_init(C.byref(cfg.c), None, C.byref(h)) == B.PIC_EINVAL and not h
    assert b"j0_target" in B.load_library().pic_last_error(None)
