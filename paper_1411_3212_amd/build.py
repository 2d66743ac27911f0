"""Compiles the HIP sources of libsj for gfx950 into ``paper_1411_3212_amd/libsj.so``."""
from __future__ import annotations

import os
import subprocess
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libsj.so"
SOURCES = ["sj_prims.hip", "sj_kernels.hip", "sj_results.hip", "sj_baseline.hip", "sj_knn.hip", "sj_api.hip", "sj_server.hip", "sj_mlp.hip", "sj_tune.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # the cell mapping relies on exact binary32 rounding of each operation
    "-ffp-contract=off",
    # no packed fp32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def build(verbose: bool = False) -> Path:
    """Always recompiles; writes the library atomically."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB.with_name(LIB.name + ".tmp%d" % os.getpid())
    cmd = [hipcc, *HIPCC_FLAGS, "-I", str(ROOT / "include"), "-o", str(tmp),
           *[str(CSRC / s) for s in SOURCES]]
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
