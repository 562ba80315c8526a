"""Register budgets and occupancy of the density kernels, from the compiler's resource
report of a device-only gfx950 build (no GPU needed).  Occupancy of the traversal kernels
is what hides the latency of their dependent node loads: a change that raises their
register count (it happened once to the persistent batch kernel, 70 -> 132 VGPRs, halving
its speed) or costs the one-sample-per-lane walks their 8 waves per SIMD (7 waves: the
paper-shaped map 10 % slower) fails here rather than on the bench."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_07571_amd", "csrc")
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


@pytest.fixture(scope="module")
def usage(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc is not installed")
    out = tmp_path_factory.mktemp("ru") / "k_density.o"
    cmd = [HIPCC, "-O3", "--offload-arch=gfx950", "-std=c++17", "-ffp-contract=off", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "hip",
           "--offload-device-only", "-c", os.path.join(CSRC, "k_density.hip"), "-o", str(out),
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"remark: \s*([A-Za-z ]+?)(?: \[[^\]]*\])?: (\d+)", line)
        if cur and m:
            kernels[cur][m.group(1).strip()] = int(m.group(2))
    return kernels


def _find(usage, pattern):
    hits = [v for k, v in usage.items() if re.search(pattern, k)]
    assert hits, pattern
    return hits


@pytest.mark.parametrize("pattern,max_vgpr,min_waves,max_scratch", [
    (r"k_densityILi1ELi1ELb0ELb0E", 64, 8, 0),     # full occlusion, scene BVH (the benchmark's kernel)
    (r"k_densityILi2ELi0ELb0ELb0E", 64, 8, 0),     # gate and exact value only
    (r"k_densityILi1ELi1ELb1ELb0E", 64, 8, 0),     # one BVH per mesh (posed maps)
    # the persistent batch kernel keeps one 8-byte value in scratch: stored at entry,
    # read once per work item, outside the walk
    (r"k_density_queueILi1ELi(64|128|256)E", 64, 8, 16),
    (r"k_zbuffer", 64, 8, 0),
])
def test_register_budget(usage, pattern, max_vgpr, min_waves, max_scratch):
    for ru in _find(usage, pattern):
        assert ru["VGPRs"] <= max_vgpr, ru
        assert ru["Occupancy"] >= min_waves, ru
        assert ru.get("ScratchSize", 0) <= max_scratch, ru
