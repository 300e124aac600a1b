"""Build of libqpat.so (HIP for gfx950), in-tree next to this file.

`build()` always recompiles; it runs on machines without a GPU because hipcc
cross-compiles for gfx950.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqpat.so")
SOURCES = ["kernels.hip", "plan.cpp", "recon.hip", "recon.cpp", "k3d.hip", "plan3d.cpp", "optical.hip", "optical.cpp", "probe.hip"]

# -packed-fp32-ops keeps the compiler from emitting packed FP32 VALU ops.
HIP_FLAGS = ["-O3", "--offload-arch=gfx950", "-mcode-object-version=5", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Per-source compiler flags (none at present).
SOURCE_FLAGS: dict[str, list[str]] = {}
# roctx ranges around the entry points (shown by rocprofv3 --marker-trace)
LINK_LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libqpat)")


def _run(cmd: list[str], verbose: bool) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{r.stdout}\n{r.stderr}")


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source to an object (in parallel: the sources are
    independent), then link the shared library in place of the old one."""
    cc = hipcc()
    jobs = jobs or min(len(SOURCES), max(1, min(os.cpu_count() or 1, 8)))
    with tempfile.TemporaryDirectory(prefix="qpat_build_") as tmpd:
        objs = [os.path.join(tmpd, src + ".o") for src in SOURCES]   # x.hip and x.cpp both exist
        cmds = [[cc, *HIP_FLAGS, *SOURCE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
                for src, obj in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp"
        _run([cc, *HIP_FLAGS, "-shared", *objs, "-o", tmp, *LINK_LIBS], verbose)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
