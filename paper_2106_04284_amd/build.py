"""Builds libllama_mi355x.so in-tree: the HIP kernels for gfx950 with hipcc,
the host C++ with g++, linked by hipcc.  Run as ``python -m
paper_2106_04284_amd.build`` or through ``__graft_entry__.build()``."""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libllama_mi355x.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed-FP32 instructions are kept out of every HIP object on purpose
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + INCLUDE, "-I" + CSRC]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-I" + INCLUDE, "-I" + CSRC,
             "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]

HIP_SOURCES = ["kernels.hip"]
CXX_SOURCES = ["core.cpp", "capi.cpp", "batch.cpp", "tune.cpp", "serve.cpp", "leaves.cpp", "box.cpp", "transfer.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def _scratch_instructions(asm: str) -> dict:
    """Scratch (private memory) loads and stores per kernel in device assembly."""
    out, kernel = {}, None
    for line in asm.splitlines():
        m = re.match(r"^(_Z\S+):", line)
        if m:
            kernel = m.group(1)
            out.setdefault(kernel, 0)
            continue
        op = line.strip().split(" ", 1)[0]
        if kernel and (op.startswith("scratch_") or op.startswith("buffer_")):
            out[kernel] += 1
    return out


def _check_no_scratch(report: str, asm: str):
    """Every kernel keeps its values in registers: a kernel that spills (or
    keeps an array in scratch memory) runs many times slower, so the build
    refuses it.  `report` is hipcc's kernel-resource-usage remarks, `asm` the
    device assembly.  A private segment without a single scratch load or store
    is the compiler's reserved emergency slot (kernels whose uniform values
    spill to VGPR lanes get one), and is accepted."""
    used = _scratch_instructions(asm)
    kernel, bad = None, []
    for line in report.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            kernel = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        # the counted (Heatmap) variants are debugging tools: they may spill
        if m and int(m.group(1)) > 0 and "count_kernel" not in (kernel or "") and used.get(kernel, 1) > 0:
            bad.append(f"{kernel}: {m.group(1)} bytes of scratch per lane, {used.get(kernel, '?')} scratch accesses")
    if bad:
        raise RuntimeError("kernels use scratch memory (register spills):\n" + "\n".join(bad))


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for s in HIP_SOURCES:
        jobs.append([HIPCC] + HIP_FLAGS + ["-Rpass-analysis=kernel-resource-usage", "-c", os.path.join(CSRC, s),
                                           "-o", os.path.join(BUILD, s + ".o")])
        jobs.append([HIPCC] + HIP_FLAGS + ["--cuda-device-only", "-S", os.path.join(CSRC, s),
                                           "-o", os.path.join(BUILD, s + ".s")])
    for s in CXX_SOURCES:
        jobs.append(["g++"] + CXX_FLAGS + ["-c", os.path.join(CSRC, s), "-o", os.path.join(BUILD, s + ".o")])
    reports = {}
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if r.args[0] == HIPCC and "-c" in r.args:
                reports[r.args[r.args.index("-c") + 1]] = r.stderr
            elif verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr)
    for s in HIP_SOURCES:
        with open(os.path.join(BUILD, s + ".s")) as f:
            _check_no_scratch(reports[os.path.join(CSRC, s)], f.read())
    objs = [os.path.join(BUILD, s + ".o") for s in HIP_SOURCES + CXX_SOURCES]
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
