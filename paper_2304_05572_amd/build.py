"""Build the HIP library libhgks.so (gfx950) in-tree from csrc/ with hipcc."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = ["hgks_kernels.hip", "hgks_kernels3.hip", "hgks_stepper.hip", "hgks_capi.cpp"]
LIB = os.path.join(HERE, "libhgks.so")
ARCH = os.environ.get("HGKS_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions stay disabled: plain scalar FP32/FP64 arithmetic only. The device pass
         # honours the feature; the host pass does not know it and warns "'-packed-fp32-ops' is not a
         # recognized feature for this target (ignoring feature)" once per source, which is harmless
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-result"]


def _compile(src, verbose):
    obj = os.path.join(HERE, "csrc", "_build", os.path.splitext(src)[0] + ".o")
    os.makedirs(os.path.dirname(obj), exist_ok=True)
    cmd = ["hipcc", "-x", "hip", *FLAGS, "-c", os.path.join(HERE, "csrc", src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def build(verbose: bool = False) -> str:
    with cf.ThreadPoolExecutor(len(SRC)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SRC))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
