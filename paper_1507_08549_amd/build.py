"""Build ``libhydro.so`` (the HIP library behind include/hydro.h) in-tree for gfx950.

Each translation unit is compiled with hipcc to an object, then linked into a
shared library next to this file.  FP64 units use ``-ffp-contract=off`` (only
the explicit fused multiply-adds are fused, so the FP64 results are a fixed
sequence of IEEE operations); the FP32-bulk unit allows contraction.  Packed
FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhydro.so")
# measurement aid, kept out of the solver library (csrc/probe.h)
PROBE_LIB = os.path.join(HERE, "libhydro_probe.so")
PROBE_UNITS = {"probe.hip": []}
ARCH = os.environ.get("HYDRO_OFFLOAD_ARCH", "gfx950")

# translation unit -> extra flags
UNITS = {
    "hydro_api.hip": ["-ffp-contract=off"],
    "stage_fp64.hip": ["-ffp-contract=off"],
    "stage_fp32.hip": ["-ffp-contract=fast"],
    "reduce.hip": ["-ffp-contract=off"],
    "poisson.hip": ["-ffp-contract=off"],
    "levelset.hip": ["-ffp-contract=off"],
    "vjp_fp64.hip": [],
    "vjp_fp32.hip": [],
}


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    objdir = os.path.join(ROOT, "_build", "hydro")
    os.makedirs(objdir, exist_ok=True)
    common = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC,
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

    def compile_one(item):
        name, extra = item
        obj = os.path.join(objdir, name + ".o")
        cmd = [hipcc, *common, *extra, "-c", os.path.join(CSRC, name), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    units = list(UNITS.items()) + list(PROBE_UNITS.items())
    with ThreadPoolExecutor(max_workers=min(len(units), 8)) as ex:
        objs = dict(zip([u for u, _ in units], ex.map(compile_one, units)))
    for lib, names in ((LIB, UNITS), (PROBE_LIB, PROBE_UNITS)):
        tmp = lib + ".tmp"
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *(objs[u] for u in names)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
