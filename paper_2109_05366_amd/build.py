"""Build libgfs.so (host runtime + device library + workload kernels) for gfx950 with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgfs.so")

SOURCES = ["gfs_host.cpp", "gfs_kernels.hip", "gfs_serve.hip"]
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed fp32 instructions in the code objects
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


# a user kernel of the device API that the tests call (gopen by path, error returns)
PROBE_SRC = os.path.join(ROOT, "tests", "csrc", "gfs_api_probe.hip")
PROBE_LIB = os.path.join(ROOT, "tests", "libgfs_api_probe.so")


def _hipcc_shared(sources, out, verbose: bool) -> str:
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIP_FLAGS + ["-shared", "-I", INCLUDE, "-o", tmp] + list(sources) + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature: harmless
    noise = [ln for ln in (r.stderr or "").splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if r.returncode != 0:
        if os.path.exists(tmp):
            os.unlink(tmp)
        raise RuntimeError("hipcc failed:\n" + "\n".join(noise))
    if verbose and noise:
        print("\n".join(noise), file=sys.stderr)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Compile every source into libgfs.so, and the tests' device-API probe into
    tests/libgfs_api_probe.so (always recompiles); returns the library path."""
    _hipcc_shared([os.path.join(CSRC, s) for s in SOURCES], LIB, verbose)
    if os.path.exists(PROBE_SRC):
        _hipcc_shared([PROBE_SRC], PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
