"""Build the gfx950 HIP library libtrtlbm.so in-tree with hipcc."""
from __future__ import annotations

import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtrtlbm.so")
SOURCES = ["api.hip", "sweep.hip", "fields.hip", "probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused only within one source expression, never across
    # statements: which products fuse is then fixed by the source, not by how
    # a kernel's code is scheduled into blocks, so every sweep variant (one or
    # two columns per lane, single or batched launch, any rows per
    # wavefront) rounds each node's arithmetic identically
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-command-line-argument",
    # per-kernel register use (read back below: a sweep kernel that spills
    # registers to scratch memory fails the build)
    "-Rpass-analysis=kernel-resource-usage",
]


def spills(remarks: str) -> dict:
    """{kernel: VGPRs spilled to scratch memory} from the compiler's resource
    remarks.  (SGPR spills go to VGPR lanes, not to memory.)"""
    out, name = {}, None
    for line in remarks.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            out.setdefault(name, 0)
            continue
        m = re.search(r"remark:\s+VGPRs Spill: (\d+)", line)
        if m and name is not None:
            out[name] += int(m.group(1))
    return out


def build(verbose: bool = False) -> str:
    """Compile every HIP source into paper_2312_10318_amd/libtrtlbm.so."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libtrtlbm.so")
    spilled = {k: n for k, n in spills(r.stderr).items()
               if n > 0 and ("sweep" in k or "probe" in k)}
    if spilled:
        os.remove(tmp)
        raise RuntimeError("sweep kernels spill registers to scratch memory: %s" % spilled)
    os.replace(tmp, LIB)
    return LIB


EXAMPLE_SRC = os.path.join(HERE, "examples", "taylor_green.cpp")
EXAMPLE = os.path.join(HERE, "examples", "taylor_green")


def build_example(verbose: bool = False) -> str:
    """Compile the C-ABI example (host code only) against libtrtlbm.so."""
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-O2", "-std=c++17", EXAMPLE_SRC, "-o", EXAMPLE,
           "-L" + HERE, "-ltrtlbm", "-Wl,-rpath,$ORIGIN/.."]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building the C-ABI example")
    return EXAMPLE


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_example(verbose=True))
