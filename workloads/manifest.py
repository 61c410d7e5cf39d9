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
* serve (C5, scaled to one disk): the pool's sizes are the same lognormal (mu = ln 128 MiB,
  sigma = 1.2) clipped to [16 MiB, 4 GiB] from seed 1000005; the full 512-file pool (about
  138 GiB) does not fit the disk, so the first 64 draws of that stream form the pool (file
  j has contents seed 10000 + j) and the cache budget keeps the full design's ratio of a
  quarter of the pool. Requests: 20 000 Poisson arrivals at 200/s from SplitMix64(seed 7); request
  i takes the uniforms of outputs 2i+1 and 2i+2: the gap since the previous arrival is
  -ln(1 - u) / rate (inverse CDF) and the file is floor(u' * pool). Times are integer ns.
  Other rates reuse the same draws with every time scaled by 200 / rate.
* serve_small: pool of 16 files (mu = ln 4 MiB, clip [256 KiB, 32 MiB], seed 1000015,
  contents seed 20000 + j), 120 requests at 2000/s from seed 17, budget 16 MiB.

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


def poisson_arrivals(seed: int, n: int, rate_per_s: float, pool: int) -> List[Dict[str, int]]:
    u = _uniforms(seed, 2 * n)
    t = 0.0
    out = []
    for i in range(n):
        t += -math.log(1.0 - u[2 * i]) / rate_per_s
        out.append({"t_ns": int(round(t * 1e9)), "file": min(int(u[2 * i + 1] * pool), pool - 1)})
    return out


def build_serve(small: bool = False) -> Dict[str, object]:
    if small:
        sizes = lognormal_sizes(1000015, 16, 4 * MiB, 1.2, 256 << 10, 32 * MiB)
        files = [{"name": f"c5s_{j:03d}.bin", "seed": 20000 + j, "size": s} for j, s in enumerate(sizes)]
        return {"name": "serve_small", "budget_bytes": 16 * MiB, "rate_per_s": 2000,
                "files": files, "requests": poisson_arrivals(17, 120, 2000.0, len(files))}
    sizes = lognormal_sizes(1000005, 64, 128 * MiB, 1.2, 16 * MiB, 4 * GiB)
    files = [{"name": f"c5_{j:03d}.bin", "seed": 10000 + j, "size": s} for j, s in enumerate(sizes)]
    budget = sum(sizes) // 4 // GiB * GiB
    return {"name": "serve", "budget_bytes": budget, "rate_per_s": 200,
            "files": files, "requests": poisson_arrivals(7, 20000, 200.0, len(files))}


def scaled_arrivals(m: Dict[str, object], rate_per_s: int) -> List[int]:
    """Arrival times (ns) of a serving manifest replayed at another rate."""
    base = int(m["rate_per_s"])
    return [r["t_ns"] * base // rate_per_s for r in m["requests"]]


def manifest_path(name: str) -> str:
    return os.path.join(MANIFEST_DIR, f"{name}.json")


def load(name: str) -> Dict[str, object]:
    with open(manifest_path(name)) as fh:
        return json.load(fh)


def write_all() -> None:
    os.makedirs(MANIFEST_DIR, exist_ok=True)
    for m in (build_batch(False), build_batch(True), build_serve(False), build_serve(True)):
        with open(manifest_path(m["name"]), "w") as fh:
            json.dump(m, fh, indent=1)
            fh.write("\n")


if __name__ == "__main__":
    write_all()
    for n in ("batch", "batch_small", "serve", "serve_small"):
        m = load(n)
        tot = sum(f["size"] for f in m["files"])
        print(n, len(m["files"]), "files", round(tot / GiB, 2), "GiB")
