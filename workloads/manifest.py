"""Frozen manifests of the multi-file workloads (sizes, seeds, arrival times).

Sizes and arrival times are drawn once from SplitMix64 streams and written to JSON files
under ``workloads/manifests/``; the GPU harness and the oracle both read those files, so a
difference in floating-point libraries can never make them disagree.

* batch (C4): 64 files, size = exp(ln(128 MiB) + 1.2 z), z standard normal by Box-Muller
  on SplitMix64(seed 1000004) with u = (x >> 11) * 2**-53 (a zero u is replaced by 2**-53),
  clipped to [1 MiB, 2 GiB] and rounded down to a multiple of 8 bytes; file i has
  contents seed 100 + i.
* batch_small: the same recipe at 1/16 scale (mu = ln 8 MiB, clip [64 KiB, 128 MiB],
  12 files, seed 1000014, contents seed 200 + i) for parity tests.

Run ``python -m workloads.manifest`` to rewrite the files.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List

from . import splitmix

HERE = os.path.dirname(os.path.abspath(__file__))
MANIFEST_DIR = os.path.join(HERE, "manifests")
MiB = 1 << 20
GiB = 1 << 30


def _uniforms(seed: int, n: int) -> List[float]:
    out = []
    for k in range(1, n + 1):
        x = splitmix.output_int(seed, k)
        u = (x >> 11) * 2.0 ** -53
        out.append(u if u > 0.0 else 2.0 ** -53)
    return out


def normals(seed: int, n: int) -> List[float]:
    """n standard normals: Box-Muller cosine branch on consecutive uniform pairs."""
    u = _uniforms(seed, 2 * n)
    return [math.sqrt(-2.0 * math.log(u[2 * i])) * math.cos(2.0 * math.pi * u[2 * i + 1]) for i in range(n)]


def lognormal_sizes(seed: int, n: int, median: int, sigma: float, lo: int, hi: int) -> List[int]:
    sizes = []
    for z in normals(seed, n):
        s = math.exp(math.log(median) + sigma * z)
        s = min(max(s, lo), hi)
        sizes.append(int(s) // 8 * 8)
    return sizes


def build_batch(small: bool = False) -> Dict[str, object]:
    if small:
        sizes = lognormal_sizes(1000014, 12, 8 * MiB, 1.2, 64 << 10, 128 * MiB)
        files = [{"name": f"c4s_{i:02d}.bin", "seed": 200 + i, "size": s} for i, s in enumerate(sizes)]
        return {"name": "batch_small", "cache_bytes": 256 * MiB, "files": files}
    sizes = lognormal_sizes(1000004, 64, 128 * MiB, 1.2, 1 * MiB, 2 * GiB)
    files = [{"name": f"c4_{i:02d}.bin", "seed": 100 + i, "size": s} for i, s in enumerate(sizes)]
    return {"name": "batch", "cache_bytes": 16 * GiB, "files": files}


def manifest_path(name: str) -> str:
    return os.path.join(MANIFEST_DIR, f"{name}.json")


def load(name: str) -> Dict[str, object]:
    with open(manifest_path(name)) as fh:
        return json.load(fh)


def write_all() -> None:
    os.makedirs(MANIFEST_DIR, exist_ok=True)
    for small in (False, True):
        m = build_batch(small)
        with open(manifest_path(m["name"]), "w") as fh:
            json.dump(m, fh, indent=1)
            fh.write("\n")


if __name__ == "__main__":
    write_all()
    for n in ("batch", "batch_small"):
        m = load(n)
        tot = sum(f["size"] for f in m["files"])
        print(n, len(m["files"]), "files", round(tot / GiB, 2), "GiB")
