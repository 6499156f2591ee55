"""Compile the oracle's C direct sums into oracle/liboracle.so (gcc + OpenMP).

Test infrastructure only; the HIP library's build never touches this file.
"""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


SANITIZE_LIB = os.path.join(os.path.dirname(_HERE), "_build", "sanitize", "liboracle.so")


def build(sanitize=False) -> str:
    """sanitize: a second copy under _build/sanitize/ with AddressSanitizer and
    UndefinedBehaviorSanitizer (ORACLE_LIB_PATH points the loader at it)."""
    src = os.path.join(_HERE, "direct.c")
    out = SANITIZE_LIB if sanitize else os.path.join(_HERE, "liboracle.so")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"] \
        if sanitize else []
    cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", *san, "-o", tmp, src]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    import sys
    print(build(sanitize="--sanitize" in sys.argv))
