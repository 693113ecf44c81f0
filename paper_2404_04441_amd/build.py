"""Build libwave.so (gfx950) in-tree with hipcc.

    python -m paper_2404_04441_amd.build
"""
from __future__ import annotations

import os
import shutil
from concurrent.futures import ThreadPoolExecutor
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libwave.so")
# the benchmark's bandwidth ceilings (plain streams of the step's traffic
# shape), a library of their own: not part of libwave's interface
PROBE_LIB = os.path.join(PKG, "libwave_probe.so")
PROBE_SOURCES = ["stream_probe.hip"]
ARCH = "gfx950"

# The step-kernel templates (step_kernels.h) are instantiated in one unit per
# storage type and one for the adjoint, so the units compile in parallel.
SOURCES = ["step_f32.hip", "step_f16.hip", "step_bf16.hip", "step_f16m.hip", "step_bf16m.hip", "step_adj.hip",
           "wave_kernels.hip", "wave_static.hip", "wave_runtime.cpp"]

# Packed-FP32 instructions stay off: they are not used on purpose anywhere in
# the kernels, and the compiler would otherwise form them from float pairs.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libwave)")


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 and link libwave.so; returns its path."""
    cc = hipcc()
    objs, probe_objs, cmds = [], [], []
    build_dir = os.path.join(PKG, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES + PROBE_SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        cmd = [cc, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
               "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".hip"):
            cmd[1:1] = ["-x", "hip"]
            cmd += DEVICE_FLAGS
        cmds.append(cmd)
        (probe_objs if src in PROBE_SOURCES else objs).append(obj)
    jobs = max(1, min(len(cmds), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as pool:
        for f in [pool.submit(_run, c, verbose) for c in cmds]:
            f.result()
    for lib, parts in ((LIB, objs), (PROBE_LIB, probe_objs)):
        tmp = lib + ".tmp"
        _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + parts, verbose)
        os.replace(tmp, lib)
    return LIB


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"build failed ({res.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
