"""Builds librkmi.so for gfx950 with hipcc.

Steps: generate the right-hand-side sources of the compiled networks, compile
every .hip translation unit to an object (in parallel), link the shared
library in place next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "gen")
OBJ = os.path.join(ROOT, "_build", "obj")
LIB = os.path.join(HERE, "librkmi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Networks compiled into the library (species counts of the standard networks).
COMPILED_NETWORKS = (9, 13, 32, 53)
# Ragged batches compiled as one kernel (species counts, in order).
COMPILED_BATCHES = ((9, 13, 32, 53),)
# Networks also compiled with the energy equation (state T, Y): up to 15 species
# with the one-lane kernels, above on the group schedule.
COMPILED_THERMAL = (9, 13, 32, 53)

CXXFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Wno-unused-function", "-Wno-unused-variable",
    # packed FP32 instructions stay off (correctness on this hardware)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # every operation rounds once, in source order: results reproduce the
    # reference evaluation bit for bit
    "-ffp-contract=off",
]


def sources():
    from . import codegen, gen_crmath
    from .inputs import standard_network
    gen_crmath.generate()
    nets = [standard_network(k) for k in COMPILED_NETWORKS]
    batches = [[standard_network(k) for k in b] for b in COMPILED_BATCHES]
    thermal = [standard_network(k) for k in COMPILED_THERMAL]
    gen = codegen.generate(nets, batches=batches, thermal=thermal)
    hand = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".hip")]
    return hand + gen


def kernel_source_digest() -> str:
    """SHA-1 over every kernel source and the compile flags: identifies the
    kernels a measurement was taken on."""
    import hashlib
    h = hashlib.sha1(" ".join(CXXFLAGS).encode())
    for d in (CSRC, GEN):
        for f in sorted(os.listdir(d)):
            if f.endswith((".hip", ".hpp", ".cpp")):
                with open(os.path.join(d, f), "rb") as fh:
                    h.update(f.encode())
                    h.update(fh.read())
    return h.hexdigest()


def _compile(src: str, resource_usage: bool) -> tuple[str, str]:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    if src.endswith(".cpp"):   # host-only C++ (no device code)
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"g++ failed for {src}:\n{r.stderr}")
        return obj, r.stderr
    cmd = [HIPCC, *CXXFLAGS, "-c", src, "-o", obj]
    if resource_usage:
        cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj, r.stderr


def build(verbose: bool = False, resource_usage: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(8, os.cpu_count() or 1, len(srcs))
    objs, logs = [], []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for obj, log in ex.map(lambda s: _compile(s, resource_usage), srcs):
            objs.append(obj)
            logs.append(log)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        for log in logs:
            if log.strip():
                print(log)
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    from paper_1611_02274_amd.build import build as _b
    _b(verbose=True, resource_usage="--usage" in sys.argv)
