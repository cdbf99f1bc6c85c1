"""Build libhekan.so in-tree with hipcc for gfx950.

python -m paper_2409_07751_amd.build  [--debug]
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhekan.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["kernels.hip", "ntt.hip", "noalloc.hip", "hostmath.cpp", "ckks.cpp", "kan.cpp", "boot.cpp", "capi.cpp",
           "server.cpp"]

COMMON = ["-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-ffp-contract=off", "-I" + os.path.join(HERE, "..", "include")]
# every HIP compilation: gfx950 only, and no packed-FP32 instructions
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(debug=False, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    opt = ["-O1", "-g"] if debug else ["-O3"]

    def compile_one(src):
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        cmd = [HIPCC] + COMMON + opt + DEVICE + ["-c", path, "-o", obj]
        if src.endswith(".hip"):
            cmd[1:1] = ["-x", "hip"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
        if verbose and r.stderr.strip():
            print(r.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC"] + DEVICE + objs + ["-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(debug="--debug" in sys.argv, verbose=True))
