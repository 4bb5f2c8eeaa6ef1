"""Build the gfx950 shared library libpic1d.so in-tree (paper_1608_04601_amd/lib/).

    python -m paper_1608_04601_amd.build
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libpic1d.so")
SOURCES = [os.path.join(CSRC, "pic_kernels.hip"), os.path.join(CSRC, "pic_api.cpp"),
           os.path.join(CSRC, "mlp_kernels.hip"), os.path.join(CSRC, "mlp_api.cpp")]
ARCH = "gfx950"


def hipcc_path():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def compile_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
            # no implicit a*b+c contraction: the arithmetic is exactly as written (fused only
            # where fmaf is spelled out), so results do not change with code layout
            "-ffp-contract=off",
            # packed FP32 VALU forms are kept out of the generated code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc_path()] + compile_flags() + ["-shared"] + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libpic1d.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
