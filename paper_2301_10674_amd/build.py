"""Build ``libfsl.so`` (the gfx950 HIP library behind ``include/fsl.h``).

Run ``python -m paper_2301_10674_amd.build``; the library lands next to this
file.  Every HIP source is compiled for gfx950 only, with packed-FP32
instructions disabled.

The compiler's per-kernel resource report (``-Rpass-analysis=kernel-
resource-usage``) is kept in ``_build/kernel_resources.txt`` and checked:
the build fails if any kernel accesses a private (scratch) segment.  Every
kernel of the library keeps its values in registers -- VGPRs, and AGPRs as
the compiler's spill space, which needs no memory -- so a scratch access
means an array the compiler could not keep in registers (an index it could
not resolve at compile time, or register pressure beyond the register file),
which is a change to look at before it runs.  A kernel at the edge of the
register file may be given a segment that no instruction touches (the
register allocator's emergency slot); for every kernel that reports a
segment the device assembly is generated and searched for scratch
instructions, and only an access fails the build.  gfx950 addresses the
private segment with flat-scratch instructions (``scratch_load_*`` /
``scratch_store_*``) only; the buffer instructions that the dense kernel
issues go through its own resource descriptors over the PDF arrays and are
not counted.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfsl.so")
SOURCES = ["fsl_step.hip", "fsl_mlp.hip", "fsl_dem.hip", "fsl_api.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-result",
    "-Rpass-analysis=kernel-resource-usage",
] + os.environ.get("FSL_EXTRA_HIPCC", "").split()


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def kernel_resources(remarks: str) -> dict:
    """{kernel: {field: value}} from the compiler's resource remarks."""
    out, cur = {}, None
    for line in remarks.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        m = re.search(r"remark:\s+(.+?): (\S+) \[-Rpass-analysis", line)
        if m and cur:
            out[cur][m.group(1).strip()] = m.group(2)
    return out


def check_resources(res: dict) -> list:
    """Kernels that report a scratch segment."""
    return [k for k, v in res.items() if v.get("ScratchSize [bytes/lane]", "0") != "0"]


def scratch_accesses(src: str, kernels: list) -> dict:
    """{kernel: number of scratch instructions} in the device assembly of
    src."""
    asm = subprocess.run([hipcc(), *[f for f in HIPCC_FLAGS if not f.startswith("-Rpass")], "--offload-device-only",
                          "-S", src, "-o", "-"], capture_output=True, text=True, check=True).stdout
    out = {}
    for k in kernels:
        i = asm.find("\n" + k + ":")
        j = asm.find(".Lfunc_end", i)
        if i < 0 or j < 0:
            out[k] = -1
            continue
        out[k] = sum(1 for l in asm[i:j].splitlines()
                     if re.match(r"\s+scratch_", l))
    return out


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, table, bad = [], [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [hipcc(), *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        msgs = "\n".join(l for l in r.stderr.splitlines()
                         if "remark:" not in l and "packed-fp32-ops" not in l and l.strip()
                         and not re.match(r"^\s*\d*\s*\|", l))
        if msgs and (verbose or r.returncode):
            print(msgs, file=sys.stderr, flush=True)
        if r.returncode:
            raise subprocess.CalledProcessError(r.returncode, cmd)
        res = kernel_resources(r.stderr)
        for k, v in res.items():
            table.append("%-14s %-70s VGPR %4s AGPR %4s VGPR-spill %3s scratch %4s occupancy %s" % (
                src, k, v.get("VGPRs"), v.get("AGPRs"), v.get("VGPRs Spill"),
                v.get("ScratchSize [bytes/lane]"), v.get("Occupancy [waves/SIMD]")))
        seg = check_resources(res)
        if seg:
            for k, n in scratch_accesses(os.path.join(CSRC, src), seg).items():
                if n != 0:
                    bad.append("%s: %s (%s scratch instructions)" % (src, k, n if n > 0 else "unknown"))
                else:
                    table.append("%-14s %-70s reserves a private segment that no instruction accesses" % (src, k))
        objs.append(obj)
    with open(os.path.join(objdir, "kernel_resources.txt"), "w") as fh:
        fh.write("\n".join(table) + "\n")
    if bad:
        raise RuntimeError("kernels with a scratch (private) segment:\n  " + "\n  ".join(bad))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
