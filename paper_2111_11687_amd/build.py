"""Build the HIP library ``libnmdose.so`` in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, f)
           for f in ("nmd_kernels.hip", "nmd_api.hip", "nmd_nn.hip", "nmd_ingest.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("nmd_internal.hpp", "nmd_device.hpp")] + [
    os.path.join(HERE, "..", "include", f) for f in ("nmdose.h", "nmdose_nn.h", "nmdose_ingest.h")]
LIB = os.path.join(HERE, "libnmdose.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # FP64 atomics compile to the native global/LDS add instructions
    "-munsafe-fp-atomics",
    # keep the compiler away from packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-Wl,-rpath,/opt/rocm/lib",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into one shared library; always recompiles."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass warns that it does not know the packed-fp32 feature
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if err.strip() and verbose:
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
