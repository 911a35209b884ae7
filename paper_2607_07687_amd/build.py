"""Build libgmg.so in-tree with hipcc for gfx950 (MI355X).

    python -m paper_2607_07687_amd.build

Compiles libgmg.so (the GMG solver) and libunet.so (the U-Net warm start)
next to this file.  Always recompiles.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-local-typedef",
]


LIBS = {
    "libgmg.so": ["csrc/gmg_lib.hip"],
    "libunet.so": ["csrc/unet_lib.hip"],
}


def build_one(name, srcs, verbose=False):
    out = os.path.join(HERE, name)
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, f"-I{os.path.join(ROOT, 'include')}",
           *[os.path.join(HERE, s) for s in srcs], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines()
            if "packed-fp32-ops" not in ln]
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, out)
    return out


def build(verbose=False):
    """Compile every library; returns their paths."""
    return [build_one(name, srcs, verbose) for name, srcs in LIBS.items()]


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
