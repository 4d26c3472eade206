"""Compile the FP64 C oracle with gcc.

Test infrastructure only (see ``oracle/__init__.py``).

``liboracle.so`` is the checker the tests load: -O3 for the x86-64-v3 level
(AVX2, FMA), which every current server host runs, so the library built here
also loads on the GPU hosts.  ISO C mode keeps floating-point contraction
off, so the sums are formed in the order the source states.

``liboracle_native.so`` is built on the machine that runs it, with
-march=native, for the benchmark's CPU baseline only.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_NATIVE = os.path.join(HERE, "liboracle_native.so")


def build(force: bool = True, native: bool = False) -> str:
    out = LIB_NATIVE if native else LIB
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
        return out
    tmp = out + ".tmp"
    arch = "-march=native" if native else "-march=x86-64-v3"
    cmd = ["gcc", "-O3", arch, "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra",
           "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
