"""Build libhopfpd.so (HIP for gfx950) in-tree.

    python -m paper_1712_08226_amd.build

All device code is compiled for gfx950 only, with packed FP32 instructions
disabled (plain float code only).  The library exports the C-ABI declared in
include/hopfpd.h.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhopfpd.so")
SOURCES = ["hopf_setup.cpp", "hopf_solver.hip", "hopf_mlp.hip"]
NT_INSTANCES = list(range(1, 17))    # hopf_inst.hip is compiled once per n_pad/16


def hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object, then link the shared library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    common = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include")]
    units = [(src, os.path.splitext(src)[0], []) for src in SOURCES]
    units += [("hopf_inst.hip", f"hopf_inst_nt{k}", [f"-DHOPF_NT={k}"]) for k in NT_INSTANCES]
    objs, failed, running = [], [], []

    def reap(block):
        while running and (block or any(p.poll() is not None for _, p in running)):
            for i, (name, pr) in enumerate(running):
                if pr.poll() is not None or block:
                    out, _ = pr.communicate()
                    if pr.returncode != 0:
                        failed.append((name, out))
                    elif verbose and out.strip():
                        print(out)
                    running.pop(i)
                    break
            if block:
                continue
    for src, stem, defs in units:
        obj = os.path.join(objdir, stem + ".o")
        objs.append(obj)
        cmd = [cc] + common + defs + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        while len(running) >= jobs:
            reap(False)
            if len(running) >= jobs:
                running[0][1].wait()
        running.append((stem, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    while running:
        reap(True)
    if failed:
        msg = "\n".join(f"--- {s}\n{o}" for s, o in failed)
        raise RuntimeError("HIP build failed:\n" + msg)
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
