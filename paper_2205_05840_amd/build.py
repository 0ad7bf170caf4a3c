"""Build libndmg.so in-tree with hipcc for gfx950."""
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libndmg.so")

SOURCES = ["kernels.hip", "stencil.hip", "generic.hip", "capi.hip", "host_setup.cpp", "tuning.cpp"]
# the kernels whose launch shapes the autotuner measures: a tuning table is valid only for
# the sources it was measured on
TUNED_SOURCES = ["stencil.hip", "kernels.hip", "kernels.hpp", "reduce.hpp"]


def source_key():
    h = hashlib.sha256()
    for f in TUNED_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # packed FP32 instructions stay off in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(CSRC, "_" + os.path.splitext(s)[0] + ".o")
        lang = ["-x", "hip"] if s.endswith(".hip") else []
        key = [f'-DNDMG_SOURCE_KEY="{source_key()}"'] if s == "tuning.cpp" else []
        cmd = [hipcc] + [f for f in FLAGS if f != "-shared"] + key + ["-c"] + lang + [src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = OUT + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    for o in objs:
        os.remove(o)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
