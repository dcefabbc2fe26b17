"""Build libgapd.so (HIP for gfx950) in-tree.

Each translation unit is compiled by hipcc in parallel, then linked into
``paper_2007_16076_amd/libgapd.so``.  Packed-FP32 instructions are disabled
for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libgapd.so")
# (source, object, extra flags).  k_fr.hip is compiled once per (connectivity,
# size class) pair so its template instantiations build in parallel.
FR_PARTS = [(c, s) for c in (4, 8) for s in (32, 64, 128, 192)]
UNITS = [("k_fr.hip", f"k_fr_{c}_{s}", [f"-DGAPD_CONN={c}", f"-DGAPD_S={s}"]) for c, s in FR_PARTS] + \
        [(f, f.rsplit(".", 1)[0], []) for f in
         ("k_misc.hip", "k_naive.hip", "k_frb.hip", "k_graph.hip", "capi.cpp", "server.cpp", "graph.cpp",
          "tune.cpp")]
ARCH = os.environ.get("GAPD_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    for src, name, extra in UNITS:
        obj = os.path.join(BUILD, name + ".o")
        cmd = [hipcc()] + flags() + extra + (["-x", "hip"] if src.endswith(".cpp") else []) + \
              ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((name, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip())
        if p.returncode != 0:
            failed.append(src)
            print(text, file=sys.stderr)
        elif verbose and text:
            print(text)
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = LIB + ".tmp"
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
