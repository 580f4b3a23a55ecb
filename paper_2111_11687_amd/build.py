"""Build the HIP library ``libnmdose.so`` in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, f)
           for f in ("nmd_kernels.hip", "nmd_api.hip", "nmd_nn.hip", "nmd_ingest.hip",
                     "nmd_probe.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("nmd_internal.hpp", "nmd_device.hpp")] + [
    os.path.join(HERE, "..", "include", f) for f in ("nmdose.h", "nmdose_nn.h", "nmdose_ingest.h",
                                                  "nmdose_probe.h")]
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


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass warns that it does not know the packed-fp32 feature
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    return res.returncode, err


def build(verbose: bool = False) -> str:
    """Compile every HIP source (in parallel) and link one shared library;
    always recompiles."""
    from concurrent.futures import ThreadPoolExecutor

    tag = "%d" % os.getpid()
    objs = [os.path.join(CSRC, os.path.basename(src) + ".o" + tag) for src in SOURCES]
    cmds = [[HIPCC] + [f for f in FLAGS if f not in ("-shared",) and not f.startswith("-Wl,")]
            + ["-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
    try:
        with ThreadPoolExecutor(max_workers=min(len(cmds), 8)) as ex:
            results = list(ex.map(_run, cmds))
        for cmd, (rc, err) in zip(cmds, results):
            if verbose:
                print(" ".join(cmd), flush=True)
            if rc != 0:
                raise RuntimeError("hipcc failed:\n" + err)
            if err.strip() and verbose:
                print(err, file=sys.stderr)
        tmp = LIB + ".tmp" + tag
        rc, err = _run([HIPCC] + FLAGS + ["-o", tmp] + objs)
        if rc != 0:
            raise RuntimeError("hipcc link failed:\n" + err)
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
