"""Build the HIP library liblp.so in-tree for gfx950 (hipcc cross-compiles
without a GPU).  Run as `python -m paper_1907_02891_amd.build`.

`python -m paper_1907_02891_amd.build --sanitize` builds a second copy,
_build/sanitize/liblp.so, whose host code (argument checks, plan logic,
workspace layout, twiddle tables) carries AddressSanitizer and
UndefinedBehaviorSanitizer; the GPU code is built as usual.  It is for the
CPU test suite (LP_LIB_PATH points the binding at it); see README.md."""
import os
import shlex
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(_HERE)
LIB = os.path.join(_HERE, "liblp.so")
SOURCES = ["csrc/lp_api.cpp", "csrc/lp_kernels.hip", "csrc/lp_reproject.hip", "csrc/lp_long.hip",
           "csrc/lp_noalloc.hip", "csrc/lp_debug.hip"]

# -packed-fp32-ops: keep hipcc from forming packed FP32 vector instructions.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]


# host-side sanitizers only (each flag applies to the host compilation)
SANITIZE_FLAGS = shlex.split("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
                             "-Xarch_host -fno-sanitize-recover=all -Xarch_host -fno-omit-frame-pointer -g")
SANITIZE_LIB = os.path.join(ROOT, "_build", "sanitize", "liblp.so")


def build(verbose=False, sanitize=False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(_HERE, "csrc")]
    lib = LIB
    extra = []
    odir = os.path.join(_HERE, "csrc")
    if sanitize:
        lib = SANITIZE_LIB
        odir = os.path.dirname(lib)
        os.makedirs(odir, exist_ok=True)
        extra = SANITIZE_FLAGS
    objs, procs = [], []
    for src in SOURCES:  # compiled in parallel
        path = os.path.join(_HERE, src)
        obj = os.path.join(odir, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [hipcc, *HIP_FLAGS, *extra, *inc, *lang, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for cmd, proc in procs:
        if proc.wait() != 0:
            raise subprocess.CalledProcessError(proc.returncode, cmd)
    tmp = lib + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *extra, "-shared-libsan", "-o", tmp, *objs] \
        if sanitize else [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
