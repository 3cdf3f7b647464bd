"""Host sanitizer run: build libstiles.so with AddressSanitizer and
UndefinedBehaviorSanitizer on its host code (the symbolic analysis, the
planner, the C ABI; device code is built as usual), then run the CPU test
suite (pytest -m "not gpu") against that build.

    python paper_2501_02483_amd/sanitize.py [extra pytest arguments]

The sanitized library goes to paper_2501_02483_amd/_build/sanitize/; the
tests load it through STILES_LIBRARY, with the clang ASan runtime preloaded
into the (uninstrumented) Python process.  Leak detection is off (the
interpreter itself keeps allocations to exit); any memory error or undefined
behaviour in the host code aborts the run."""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# every -fsanitize flag applies to the host compilation only
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize=vptr", "-Xarch_host", "-fno-sanitize-recover=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]
COMMON = ["-O1", "-g", "-fPIC", "-std=c++17"]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def asan_runtime():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not libs:
        raise RuntimeError("clang ASan runtime not found under /opt/rocm/llvm")
    return libs[-1]


def build():
    os.makedirs(OUT, exist_ok=True)
    objs = []
    for src in ("analyze.cpp", "capi.cpp", "ooc.cpp"):
        obj = os.path.join(OUT, src + ".o")
        subprocess.check_call([HIPCC, "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + SAN)
        objs.append(obj)
    obj = os.path.join(OUT, "kernels.hip.o")
    subprocess.check_call([HIPCC, "-x", "hip", "-c", os.path.join(CSRC, "kernels.hip"), "-o", obj] + COMMON + DEVICE)
    objs.append(obj)
    lib = os.path.join(OUT, "libstiles.so")
    subprocess.check_call([HIPCC, "-shared", "-o", lib] + objs +
                          ["--offload-arch=gfx950", "-lamdhip64", "-shared-libasan"] + SAN)
    return lib


def main(argv):
    lib = build()
    env = dict(os.environ)
    env["STILES_LIBRARY"] = lib
    env["LD_PRELOAD"] = asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-x", "-q", "-m", "not gpu"] + argv
    print("sanitized library:", lib, flush=True)
    return subprocess.call(cmd, env=env, cwd=ROOT)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
