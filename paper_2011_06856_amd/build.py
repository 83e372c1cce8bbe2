"""Build the HIP library librlbm.so in-tree for gfx950 (hipcc cross-compiles
without a GPU)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "librlbm.so")
SOURCES = ["kernels.hip", "quadrature.cpp", "capi.cpp", "batch.cpp", "mlp.hip", "push.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions stay disabled: hipcc -O3 emits them from plain float
# code, and plain VALU FP32 is what these kernels are written for.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-unknown-warning-option"]


def build(verbose=False, out=SO, defines=()):
    """Compile the library to `out`; `defines` are extra -D flags (variants)."""
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        tag = "%d_%x" % (os.getpid(), abs(hash((out, tuple(defines)))) & 0xffffff)
        obj = os.path.join(CSRC, src.rsplit(".", 1)[0] + "." + tag + ".o")
        lang = ["-x", "hip"]
        cmd = [HIPCC] + FLAGS + ["-D" + d for d in defines] + lang + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
