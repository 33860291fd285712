"""Build the library's HIP sources as host code (``libfsl_emu.so``) for CPU
tests of the kernels (see hip/hip_runtime.h for the execution model).

The sources are copied into ``_build/`` with two mechanical rewrites that
plain C++ needs -- kernel launches ``k<<<grid, block, shmem, stream>>>(a, ...)``
become ``hipemu::launch(hipemu::cfg(grid, block, shmem, stream), k, a, ...)``,
and the empty register-tie statements ``asm volatile("" : "+v"(x))`` (a
scheduling hint with no instruction) become ``(void)(x)`` -- and compiled with
clang++ (which knows _Float16 and vector extensions on the host) with
UBSan's checks, array bounds included, trapping on the first finding.
Nothing else changes: the kernels run as written.

    python tests/hostemu/build.py [--asan]
"""
from __future__ import annotations

import glob
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2301_10674_amd", "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(OUT, "libfsl_emu.so")
CLANG = "/opt/rocm/llvm/bin/clang++"
SOURCES = ["fsl_step.hip", "fsl_mlp.hip", "fsl_dem.hip", "fsl_api.hip"]
HEADERS = ["fsl_device.h", "fsl_kernels.h", "fsl_mlp.h"]


def rewrite_launches(src: str) -> str:
    out, pos = [], 0
    while True:
        k = src.find("<<<", pos)
        if k < 0:
            out.append(src[pos:])
            return "".join(out)
        # callee: identifier with optional template arguments, scanned backwards
        j = k
        if src[j - 1] == ">":
            depth, j = 0, j - 1
            while True:
                if src[j] == ">":
                    depth += 1
                elif src[j] == "<":
                    depth -= 1
                    if depth == 0:
                        break
                j -= 1
        while j > 0 and (src[j - 1].isalnum() or src[j - 1] in "_:"):
            j -= 1
        callee = src[j:k]
        e = src.find(">>>", k)
        cfg = src[k + 3:e]
        p = e + 3
        while src[p].isspace():
            p += 1
        assert src[p] == "(", src[j:p + 20]
        q = p + 1
        while src[q].isspace():
            q += 1
        sep = "" if src[q] == ")" else ", "
        out.append(src[pos:j])
        out.append("hipemu::launch(hipemu::cfg(%s), %s%s" % (cfg, callee, sep))
        pos = p + 1


def rewrite(src: str) -> str:
    src = re.sub(r'asm\s+volatile\s*\(\s*""\s*:\s*"\+v"\s*\(\s*(\w+)\s*\)\s*\)\s*;', r"(void)(\1);", src)
    src = src.replace('#include "../../include/fsl.h"', '#include "fsl.h"')
    return rewrite_launches(src)


def build(asan: bool = False) -> str:
    sdir = os.path.join(OUT, "src")
    os.makedirs(sdir, exist_ok=True)
    for f in SOURCES + HEADERS:
        text = open(os.path.join(CSRC, f)).read()
        with open(os.path.join(sdir, f.replace(".hip", ".cpp")), "w") as fh:
            fh.write(rewrite(text))
    san = ["-fsanitize=undefined,bounds", "-fno-sanitize-recover=all", "-fno-sanitize=function,vptr"]
    if asan:
        san = ["-fsanitize=address"] + san
    flags = ["-x", "c++", "-std=c++17", "-O1", "-g", "-fPIC", "-ffp-contract=off", "-Wno-unused-value",
             "-Wno-unknown-attributes", "-I" + HERE, "-I" + sdir, "-I" + os.path.join(ROOT, "include")] + san
    objs = []
    for f in [os.path.join(sdir, s.replace(".hip", ".cpp")) for s in SOURCES] + [os.path.join(HERE, "hostemu.cpp")]:
        obj = os.path.join(OUT, os.path.basename(f) + ".o")
        subprocess.run([CLANG, *flags, "-c", f, "-o", obj], check=True)
        objs.append(obj)
    lib = LIB if not asan else LIB.replace(".so", "_asan.so")
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux"))[-1]
    # -Bsymbolic: the library's own hip* stand-ins serve its calls even in a
    # process that has the real HIP runtime loaded (the GPU comparison test)
    subprocess.run([CLANG, "-shared", "-fPIC", *san, "-shared-libsan", "-Wl,-Bsymbolic", "-Wl,-rpath," + rt, *objs,
                    "-o", lib],
                   check=True)
    return lib


if __name__ == "__main__":
    print(build(asan="--asan" in sys.argv))
