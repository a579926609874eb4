"""Build libevis.so (all HIP sources, gfx950) in-tree with hipcc.

Usage: python -m paper_2607_08098_amd.build  (or build() from Python).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libevis.so")

SOURCES = ["evis_api.cpp", "evis_tile.hip", "evis_tile_splat.hip", "evis_tile_noise.hip",
           "evis_events.hip", "evis_soft.hip", "evis_voxel.hip"]

# -ffp-contract=off and correctly rounded division: every float32 operation of
# the event path is one IEEE operation rounded to nearest, as written.
# Packed FP32 instructions are kept off.
HIP_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-gpu-rdc", "-Wno-unused-result", "-Wno-unused-value",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build_id() -> str:
    """Hash of every source, the public header and the flags: names this
    build in the library's tuning-cache keys."""
    import hashlib
    h = hashlib.sha256(" ".join(HIP_FLAGS).encode())
    for name in sorted(os.listdir(CSRC)) + ["evis.h"]:
        path = os.path.join(INCLUDE if name == "evis.h" else CSRC, name)
        if os.path.isfile(path) and name.endswith((".h", ".hip", ".cpp")):
            h.update(name.encode())
            with open(path, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source to an object, link libevis.so; returns its path."""
    objdir = os.path.join(PKG, "_build")
    bid = build_id()
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        cmd = [hipcc(), "-x", "hip", "-c", path, "-o", obj, "-I", INCLUDE, "-I", CSRC,
               f'-DEVIS_BUILD_ID="{bid}"'] + HIP_FLAGS
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    while procs:
        _wait(procs.pop(0))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + ["--offload-arch=gfx950", "-fPIC"]
    if verbose:
        print(" ".join(cmd), flush=True)
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if out.returncode != 0:
        raise RuntimeError("link failed:\n" + out.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n" + out.decode(errors="replace"))
    text = out.decode(errors="replace").strip()
    lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if lines:
        print("\n".join(lines), file=sys.stderr)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
