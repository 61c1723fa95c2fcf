"""Build the HIP engine into ``paper_1108_1954_amd/libpic1d.so`` for gfx950.

Run ``python -m paper_1108_1954_amd.build`` (or ``__graft_entry__.build()``).
It always recompiles.  hipcc cross-compiles, so no GPU is needed to build.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("pic_kernels.hip", "pic_solve.hip", "pic_sort.hip", "pic_loader.hip", "pic_phase.hip", "pic_probe.hip", "pic_tune.hip", "pic_runtime.hip")]
LIB = os.path.join(HERE, "libpic1d.so")
ARCH = os.environ.get("PIC1D_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",                 # every FMA in the kernels is explicit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # kernel arguments preloaded into SGPRs at wave launch, so a launch's first
    # dependent load (work item, run descriptor, gather table) goes out without
    # waiting for a scalar load of its arguments (1-2% on launches of 10-30 us)
    "-mllvm", "-amdgpu-kernarg-preload-count=16",
    "-Wall",
    f"-I{os.path.join(ROOT, 'include')}",
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines()
            if "packed-fp32-ops" not in ln and ln.strip()]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs), flush=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
