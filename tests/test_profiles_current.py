"""The committed rocprofv3 summaries under profiles/ were taken on the kernel sources in the
tree: each records the first 16 hex digits of the SHA-256 of the source it measured, and
bench.py takes its HBM traffic from the counter summaries only when that hash matches."""
import glob
import hashlib
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = {"pic": os.path.join(ROOT, "paper_1608_04601_amd", "csrc", "pic_kernels.hip"),
           "mlp": os.path.join(ROOT, "paper_1608_04601_amd", "csrc", "mlp_kernels.hip")}


def _sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def test_profiles_name_the_current_kernel_sources():
    current = {k: _sha(p) for k, p in SOURCES.items()}
    checked = 0
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        text = open(path).read()
        m = re.search(r"kernel_source_sha[^:\n]*:\s*([0-9a-f]{16})", text)
        if not m:
            continue
        src = "mlp" if os.path.basename(path).startswith(("forward_fused", "gemm")) else "pic"
        assert m.group(1) == current[src], (os.path.basename(path), m.group(1), current[src])
        checked += 1
    assert checked >= 8


def test_bench_finds_measured_traffic_for_each_workload():
    for workload, kernel in (("large", "pass_dyn_kernel"), ("production", "pass_kernel"),
                             ("sweep", "pass_batch_kernel")):
        bpps = bench.stored_traffic(workload, kernel)
        assert bpps is not None and 20.0 < bpps < 36.0, (workload, bpps)
