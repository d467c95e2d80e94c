"""Host-side logic of bench.py that needs no GPU: the traffic file is used
only while the sources of the kernel it describes are unchanged, and the
bytes of a profiler id made of several HIP kernels are their dispatch-weighted
mean."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write(tmp_path, hashes, kernels):
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps({"source_sha256_16": hashes, "kernels": kernels}))
    return str(p)


def test_traffic_requires_unchanged_kernel_sources(tmp_path):
    now = bench._file_hashes()
    ks = {"gemm_tn_kernel": {"hbm_bytes_per_launch": 100.0, "dispatches": 4}}
    assert bench._traffic("gram", _write(tmp_path, now, ks)) == 100.0
    stale = dict(now, **{"dense.hip": "0" * 16})
    assert bench._traffic("gram", _write(tmp_path, stale, ks)) is None
    # a change to a file the kernel does not depend on keeps the figure
    other = dict(now, **{"tridiag.hip": "0" * 16})
    assert bench._traffic("gram", _write(tmp_path, other, ks)) == 100.0
    assert bench._traffic("gram", str(tmp_path / "missing.json")) is None


def test_traffic_weights_kernels_by_dispatches(tmp_path):
    now = bench._file_hashes()
    ks = {"mg3_post1_kernel": {"hbm_bytes_per_launch": 30.0, "dispatches": 10},
          "mg3_post2_kernel": {"hbm_bytes_per_launch": 10.0, "dispatches": 30}}
    assert abs(bench._traffic("mg_up", _write(tmp_path, now, ks)) - 15.0) < 1e-12


def test_kernel_sources_name_the_defining_file_and_headers():
    src = bench._kernel_sources("mg3_pre_kernel")
    assert "mg3.hip" in src and "sts_internal.h" in src and "include/sts.h" in src
    assert "dense.hip" not in src


def test_profiler_ids_name_kernels_that_exist():
    """Every HIP kernel bench.py maps to a profiler id is defined in the
    library sources, so a renamed kernel cannot silently drop its traffic
    and time from the report."""
    import re
    defined = set()
    for fn in os.listdir(bench.CSRC):
        if fn.endswith((".hip", ".h")):
            with open(os.path.join(bench.CSRC, fn)) as fh:
                text = fh.read()
            defined |= set(re.findall(
                r"__global__\s+(?:__launch_bounds__\([^)]*\)\s+)?void\s+(\w+)\s*\(", text))
    assert "gemm_nn_sub4_kernel" in defined and "mg3_post_kernel" in defined
    missing = {pid: [k for k in ks if k not in defined] for pid, ks in bench.HIP_KERNELS.items()}
    assert not any(missing.values()), missing
