"""Compile the HIP library (libmlmc.so) for gfx950 with hipcc, in-tree."""
import concurrent.futures
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmlmc.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")

SOURCES = [
    "kernels_vec.hip",
    "kernels_poisson.hip",
    "kernels_wilson.hip",
    "kernels_krylov.hip",
    "kernels_varcoef.hip",
    "kernels_nn.hip",
    "kernels_csr.hip",
    "kernels_defl.hip",
    "kernels_group.hip",
    "context.cpp",
    "context_complex.cpp",
    "context_nn.cpp",
    "context_csr.cpp",
    "context_defl.cpp",
    "context_export.cpp",
    "estimator.cpp",
    "capi.cpp",
    "noalloc.cpp",
    "group.cpp",
]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src, hipcc):
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc, "-x", "hip", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(jobs=8):
    """Compile every source and link paper_2108_11281_amd/libmlmc.so."""
    hipcc = _hipcc()
    os.makedirs(BUILD_DIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, hipcc), SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
