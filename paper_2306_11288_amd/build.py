"""Compile libqed.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2306_11288_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqed.so")
SOURCES = ["qed_abi.cpp", "qed_tables.hip", "qed_kernels.hip", "qed_mlp.hip", "qed_detector.hip", "qed_fdtd.hip", "qed_deposit.hip", "qed_noalloc.hip",
           "qed_sort.hip", "qed_brems.hip"]
ARCH = os.environ.get("QED_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return h


# Particle kernels: no machine-level loop-invariant code motion.  Hoisting the FP64 / FP32
# constants of the inlined math out of the per-event loops keeps dozens of them live in
# registers for the whole kernel and halves the occupancy; rematerialising them in the
# loop costs a few scalar moves.
EXTRA = {"qed_kernels.hip": ["-mllvm", "-disable-machine-licm"], "qed_mlp.hip": ["-mllvm", "-disable-machine-licm"]}


def build(verbose: bool = False) -> str:
    """Always recompiles (a build check must see the current sources)."""
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
              # keep packed-FP32 instructions (v_pk_*_f32) out of the generated code
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-result"]
    procs = []
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"]
        cmd = [hipcc()] + lang + common + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    errs = []
    for src, p in procs:
        out, _ = p.communicate()
        txt = out.decode(errors="replace")
        if p.returncode != 0:
            errs.append(f"--- {src}\n{txt}")
        elif verbose and txt.strip():
            print(txt)
    if errs:
        raise RuntimeError("libqed build failed:\n" + "\n".join(errs))
    tmp = LIB + ".tmp"
    subprocess.check_call([hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
