"""Compile the HIP sources of the package into liblbsoft.so and the copy
probe into libhbmprobe.so (gfx950).

hipcc builds device code for gfx950 only.  Packed FP32 instructions are
disabled for the device code (the flag is meaningless for the host pass,
which warns about it).
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblbsoft.so")
PROBE_LIB = os.path.join(HERE, "libhbmprobe.so")
PROBE_SOURCES = [os.path.join(CSRC, "hbm_probe.hip")]
SOURCES = [os.path.join(CSRC, f) for f in ("lb_kernels.hip", "lb_engine.hip", "lb_runtime.hip", "lb_pool.hip", "lb_init_spec.hip", "lb_moment.hip", "lb_split.hip", "lb_noalloc.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", f"-I{INCLUDE}", f"-I{CSRC}"]


def _compile(sources, lib, verbose):
    tmp = lib + f".tmp{os.getpid()}"
    cmd = [HIPCC, *FLAGS, *sources, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 feature; drop that noise
    noise = "is not a recognized feature for this target"
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines() if noise not in ln]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """liblbsoft.so (the library) and libhbmprobe.so (the copy-ceiling probe
    the benchmark runs beside it)."""
    _compile(PROBE_SOURCES, PROBE_LIB, verbose)
    return _compile(SOURCES, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
