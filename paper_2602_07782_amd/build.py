"""Build the HIP library (gfx950) in-tree: paper_2602_07782_amd/libtabi_hip.so.

With --phase-clock, a diagnostic copy (libtabi_hip_phase.so) whose
fold-and-push kernel records per-phase clock sums (TABI_PHASE_CLOCK)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libtabi_hip.so")
OUT_PHASE = os.path.join(HERE, "libtabi_hip_phase.so")
SOURCES = ["prep.hip", "prerot.hip", "profile.hip", "pack.hip", "api.cpp", "serve.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
         # no packed fp32 instructions in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]
# per-source flags.  The fold-and-push kernel runs at 128 VGPRs (16 wavefronts
# per workgroup): machine loop-invariant code motion hoists per-lane
# constants and addresses out of its row loop, which then spills VGPRs to
# scratch inside the loop (each reload waits on every outstanding memory
# operation).  Without that pass it spills none (fold-and-push 251 -> 236 us
# on 2,000 charts).
SOURCE_FLAGS = {"pack.hip": ["-mllvm", "-disable-machine-licm"]}


def build(verbose: bool = False, phase_clock: bool = False) -> str:
    objdir = os.path.join(HERE, "_build_phase" if phase_clock else "_build")
    out = OUT_PHASE if phase_clock else OUT
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".", "_") + ".o")
        cmd = [HIPCC, *FLAGS, *SOURCE_FLAGS.get(src, []),
               *(["-DTABI_PHASE_CLOCK"] if phase_clock else []), "-x", "hip", "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, phase_clock="--phase-clock" in sys.argv))
