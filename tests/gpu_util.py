"""Helpers shared by the GPU tests: expected values from the oracle, trace decoding."""
from __future__ import annotations

import os

import numpy as np

from oracle import data as odata
from workloads import configs

_ACTIONS = {0: "FREE", 1: "SKIP", 2: "CLEAR", 3: "EVICT"}
NONE32 = 0xFFFFFFFF


def expected(wl, path, blocks=None):
    """(consumer output, delivered bytes per block) from the oracle."""
    if wl.consumer == configs.CONSUMER_CHECKSUM:
        out = odata.block_checksums(path, wl.offsets, wl.read_size, blocks)
    else:
        out = odata.block_histograms(path, wl.offsets, wl.read_size, blocks)
    size = os.path.getsize(path)
    o = wl.offsets.astype(np.int64)
    deliv = np.maximum(np.minimum(o + wl.read_size, size) - o, 0).sum(axis=1)
    return out, deliv


def decode(ev: np.ndarray):
    """Device trace records -> the oracle's event tuples."""
    out = []
    for r in ev:
        op = int(r["op"])
        blk, f, p, fr, a, b = (int(r["block"]), int(r["file"]), int(r["page"]), int(r["frame"]),
                              int(r["a"]), int(r["b"]))
        if op == 1:
            out.append(("HIT", blk, f, p, fr))
        elif op == 2:
            out.append(("JOIN", blk, f, p, fr))
        elif op == 3:
            out.append(("MISS", blk, f, p, b & 0xFFFFFFFF, a))   # b: window start | req << 32
        elif op == 4:
            act = _ACTIONS[a & 0xFF]
            x = a >> 8            # victim's prefetched mark | what the hand found << 1
            if act == "EVICT":
                out.append(("HAND", b, fr, act, f, p, x & 1, x >> 1))
            else:
                out.append(("HAND", b, fr, act, -1, -1, 0, x >> 1))
        elif op == 5:
            out.append(("ALLOC", f, p, fr, a))
        elif op == 6:
            out.append(("REQ", f, p, a))
        elif op == 7:
            out.append(("NOFRAME", blk, f, p))
        elif op == 9:
            out.append(("ADV", blk, f, p, b, a))
        else:
            raise ValueError(f"unknown trace op {op}")
    return out


def canon(events):
    """Order-insensitive within one miss (or asynchronous window): hand visits by ticket,
    allocations by page."""
    out = []
    seg = None

    def flush():
        nonlocal seg
        if seg is not None:
            out.append((seg[0], tuple(sorted(seg[1], key=lambda e: e[1])), tuple(sorted(seg[2])),
                        tuple(seg[3]), seg[4]))
            seg = None

    for e in events:
        k = e[0]
        if k in ("HIT", "JOIN"):
            flush()
            out.append(e)
        elif k in ("MISS", "ADV"):
            flush()
            seg = [e, [], [], [], None]
        elif k == "HAND":
            seg[1].append(e)
        elif k == "ALLOC":
            seg[2].append(e)
        elif k == "NOFRAME":
            seg[3].append(e)
        elif k == "REQ":
            seg[4] = e
            flush()
    flush()
    return out


def decode_replay(ev: np.ndarray):
    """Device trace records -> the tuples oracle.replay takes (tickets and blocks kept)."""
    out = []
    for r in ev:
        op = int(r["op"])
        blk, f, p, fr, a, b = (int(r["block"]), int(r["file"]), int(r["page"]), int(r["frame"]),
                              int(r["a"]), int(r["b"]))
        if op == 3:
            out.append(("MISS", blk, f, p, b & 0xFFFFFFFF, a, fr, max(1, b >> 32)))
        elif op == 4:
            act = _ACTIONS[a & 0xFF]
            x = a >> 8
            if act == "EVICT":
                out.append(("HAND", b, fr, act, f, p, x & 1, x >> 1, blk))
            else:
                out.append(("HAND", b, fr, act, -1, -1, 0, x >> 1, blk))
        elif op == 5:
            out.append(("ALLOC", blk, f, p, fr, a, b))
        elif op == 6:
            out.append(("REQ", blk, f, p, a))
        elif op == 7:
            out.append(("NOFRAME", blk, f, p))
    return out
