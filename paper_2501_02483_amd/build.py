"""Build libstiles.so (HIP for gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libstiles.so")
GEN_LIB = os.path.join(HERE, "libstiles_gen.so")
SOURCES = ["analyze.cpp", "capi.cpp", "ooc.cpp", "kernels.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function"]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose=False):
    """Compile every source (always) and link the shared library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        if src.endswith(".hip"):
            cmd = [HIPCC, "-x", "hip", "-c", path, "-o", obj] + COMMON + DEVICE
        else:
            cmd = [HIPCC, "-c", path, "-o", obj] + COMMON
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-o", tmp] + objs + ["--offload-arch=gfx950", "-lamdhip64"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # device-side synthetic input generator: a library of its own
    gobj = os.path.join(objdir, "gen.hip.o")
    cmd = [HIPCC, "-x", "hip", "-c", os.path.join(CSRC, "gen.hip"), "-o", gobj] + COMMON + DEVICE
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    tmp = GEN_LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "-shared", "-o", tmp, gobj, "--offload-arch=gfx950", "-lamdhip64"])
    os.replace(tmp, GEN_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
