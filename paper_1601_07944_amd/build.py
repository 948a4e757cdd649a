"""Build libdgmi.so (HIP kernels + C ABI) in-tree with hipcc for gfx950.

Every source compiles to its own object in parallel (the kernels are split
into one translation unit per polynomial order); the objects are then linked
into paper_1601_07944_amd/libdgmi.so.
"""
from __future__ import annotations

import hashlib
import json
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build", "obj")
LIB = os.path.join(HERE, "libdgmi.so")
# written beside the library by build(): the hash of the sources and flags it
# was compiled from
STAMP = LIB + ".sources.json"
SOURCES = [
    "dg_kernels_p1.hip",
    "dg_kernels_p2.hip",
    "dg_kernels_p3.hip",
    "dg_kernels_p4.hip",
    "dg_kernels_p5.hip",
    "dg_kernels_f32.hip",
    "dg_kernels.hip",
    "dg_api.cpp",
    "dg_tables.cpp",
]

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # fused multiply-adds only within one source expression (or written as
    # fma()): the same expression then rounds the same way in every kernel
    # that inlines it, which the bitwise-equality guarantees rely on
    "-ffp-contract=on",
    # matrix-core instructions keep their operands and results in the
    # ordinary vector registers (no copies through the accumulation registers)
    "-mllvm",
    "-amdgpu-mfma-vgpr-form",
    # packed FP32 instructions stay off: plain scalar/float2 code only
    "-Xclang",
    "-target-feature",
    "-Xclang",
    "-packed-fp32-ops",
]

# per-file additions: the one-lane FP32 stage kernels schedule their memory
# instructions into clauses (measured faster there for p >= 2, not for p = 1 or
# the other kernels)
FILE_FLAGS = {
    "dg_kernels_f32.hip": ["-mllvm", "-amdgpu-sched-strategy=max-memory-clause"],
}


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def source_files():
    """Every file the library is compiled from: the kernel and host sources
    under csrc/ and the public header."""
    files = sorted(
        os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".h", ".hip", ".cpp"))
    )
    return files + [os.path.join(ROOT, "include", "dg.h")]


def source_hash() -> str:
    """sha256 (first 16 hex digits) of the library's sources and compiler
    flags; build() records it beside libdgmi.so."""
    h = hashlib.sha256()
    for f in source_files():
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    h.update(json.dumps([FLAGS, FILE_FLAGS, SOURCES]).encode())
    return h.hexdigest()[:16]


def built_hash():
    """The source hash libdgmi.so was built from, or None (no library, or
    no record of its sources)."""
    if not os.path.exists(LIB) or not os.path.exists(STAMP):
        return None
    try:
        with open(STAMP) as f:
            return json.load(f).get("source_sha256_16")
    except (OSError, ValueError):
        return None


def build(verbose: bool = False, extra=(), jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    digest = source_hash()

    def compile_one(src):
        obj = os.path.join(OBJ, src + ".o")
        cmd = [_hipcc(), *FLAGS, *FILE_FLAGS.get(src, []), *extra, *inc, "-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        if verbose and r.stderr:
            print(r.stderr, flush=True)
        return obj

    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    if os.path.exists(STAMP):
        os.remove(STAMP)
    os.replace(tmp, LIB)
    # extra flags make a library that no longer matches the plain sources
    rec = {"source_sha256_16": digest if not extra else None, "extra_flags": list(extra)}
    with open(STAMP, "w") as f:
        json.dump(rec, f)
    return LIB


def ensure_built() -> str:
    """Build libdgmi.so unless the library present was built from exactly
    the current sources and flags (the hash recorded beside it by build());
    a library without that record, or from other sources, is rebuilt."""
    if built_hash() == source_hash():
        return LIB
    print(f"[build] libdgmi.so missing or stale (sources {source_hash()}, built {built_hash()}): rebuilding",
          file=sys.stderr, flush=True)
    return build()


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, extra=[a for a in sys.argv[1:] if a != "-v"]))
