"""Builds libgazemap.so (gfx950) in-tree from csrc/ with hipcc; the host-only BVH
builder is compiled with g++.  Run as a module or through __graft_entry__.build()."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgazemap.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HIP_FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall"]
HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
              "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall"]

HIP_SOURCES = ["k_sampler.hip", "k_scan.hip", "k_density.hip", "k_field.hip", "capi.cpp", "field_api.cpp", "batch_api.cpp",
               "map_api.cpp", "export_api.cpp",
               "zbuffer_api.cpp", "noalloc_api.cpp"]
HOST_SOURCES = ["bvh_build.cpp", "mesh_topology.cpp"]
# per-file flags: the field kernels keep matrix-core results in ordinary vector registers
# (no copies out of the accumulation registers before the bias/ReLU/convert steps)
EXTRA_FLAGS = {"k_field.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def _compile(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r.stderr


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    jobs = []
    for src in HIP_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        jobs.append([HIPCC, *HIP_FLAGS, *EXTRA_FLAGS.get(src, []), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", o])
    for src in HOST_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        jobs.append(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", o])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for err in ex.map(_compile, jobs):
            if verbose and err.strip():
                print(err, file=sys.stderr)
    objs = [os.path.join(OBJ, s + ".o") for s in HIP_SOURCES + HOST_SOURCES]
    tmp = LIB + ".tmp"
    _compile([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
