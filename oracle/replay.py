"""Replay of a concurrent run's policy trace against the model's rules.

Test infrastructure only (see the package docstring).

In a concurrent run the order in which threadblocks miss, allocate and evict is decided
by the hardware (Sec. 3.2: threadblocks run in a non-deterministic order), so there is
no single predicted trace. The trace is instead checked against the rules along the
run's own linearization, the method Sec. 3.3 uses when it records the GPU's I/O trace
and replays it on the CPU:

* clock: every hand ticket is taken once; frame histories rebuilt in ticket order must
  be consistent -- a FREE visit finds a frame that never held a page, an EVICT names
  exactly the page the frame received at its previous claim, every claim is followed by
  an allocation with the same ticket, no page is held by two frames at once, and the
  eviction order is the EVICT records sorted by ticket;
* readahead: the misses of a file are logged under its miss lock, so their record order
  is the order the detector saw them. Replaying the stream table and the recent-miss
  ring gives the exact window of every decision taken by a stream zone or by the
  aggregate (near-miss) rule, and the exact near count; a decision by the context rule
  depends on which pages were cached at that instant, so only its shape is checked
  (it starts at the missed page, and its length is 1, W0 or an even 2h <= cap);
* requests: each block's own records are in program order, so every miss is followed by
  that block's allocations and one request, which must cover exactly the contiguous run
  of allocated pages inside the window, starting with the demanded page.

Events are tuples:
  ("MISS", block, file, page, ws, wn, near)
  ("HAND", ticket, frame, action, vfile, vpage, vra, block)
  ("ALLOC", block, file, page, frame, ra, ticket)
  ("REQ", block, file, first, npages)
  ("NOFRAME", block, file, page)
"""
from __future__ import annotations

from collections import defaultdict
from typing import Dict, List, Tuple

from .policy import NEAR_MIN, NEAR_PAGES, RECENT


class ReplayError(AssertionError):
    pass


def _check(cond: bool, msg: str) -> None:
    if not cond:
        raise ReplayError(msg)


def replay_clock(events, nframes: int) -> Dict[str, object]:
    """Frame histories in hand-ticket order; returns eviction order and counts."""
    hands = sorted((e for e in events if e[0] == "HAND"), key=lambda e: e[1])
    allocs = {e[6]: e for e in events if e[0] == "ALLOC"}
    tickets = [e[1] for e in hands]
    _check(len(set(tickets)) == len(tickets), "a hand ticket was taken twice")
    if tickets:
        _check(tickets == list(range(tickets[0], tickets[0] + len(tickets))),
               "hand tickets are not contiguous (trace truncated?)")
    occupant: Dict[int, Tuple[int, int, int]] = {}      # frame -> (file, page, ra at alloc)
    where: Dict[Tuple[int, int], int] = {}              # (file, page) -> frame
    evictions: List[Tuple[int, int, int, int]] = []     # (ticket, frame, file, page)
    wasted = 0
    for e in hands:
        _, t, f, act, vf, vp, vra, _blk = e
        _check(f == t % nframes, f"ticket {t} visited frame {f}, expected {t % nframes}")
        if act == "FREE":
            _check(f not in occupant, f"FREE visit at ticket {t} but frame {f} holds {occupant.get(f)}")
        elif act == "EVICT":
            _check(f in occupant, f"EVICT at ticket {t} of empty frame {f}")
            of, op, ora = occupant[f]
            _check((of, op) == (vf, vp), f"EVICT at ticket {t}: frame {f} holds {(of, op)}, trace says {(vf, vp)}")
            _check(vra <= ora, f"EVICT at ticket {t}: prefetched mark set on a demanded page")
            del occupant[f]
            del where[(of, op)]
            evictions.append((t, f, vf, vp))
            wasted += vra
        if act in ("FREE", "EVICT"):
            _check(t in allocs, f"claim at ticket {t} (frame {f}) has no allocation")
            a = allocs[t]
            _, _blk2, af, ap, aframe, ara, _ = a
            _check(aframe == f, f"allocation at ticket {t} names frame {aframe}, hand was at {f}")
            _check((af, ap) not in where, f"page {(af, ap)} held by frames {where.get((af, ap))} and {f}")
            occupant[f] = (af, ap, ara)
            where[(af, ap)] = f
        else:
            _check(t not in allocs, f"ticket {t} was a {act} visit but has an allocation")
    _check(len(allocs) == sum(1 for e in hands if e[3] in ("FREE", "EVICT")),
           "allocations without a matching claim")
    return {"evictions": evictions, "wasted_pages": wasted, "allocations": len(allocs),
            "resident": len(occupant)}


def replay_readahead(events, ra_init: int, ra_cap: int, streams: int,
                     files: Dict[int, int], page_size: int, advice: Dict[int, str] = None):
    """Replay every file's miss decisions in lock (record) order."""
    advice = advice or {}
    state = {}
    checked_exact = 0
    checked_shape = 0
    for e in events:
        if e[0] != "MISS":
            continue
        _, blk, fid, p, ws, wn, near = e
        npages = (files[fid] + page_size - 1) // page_size
        if ra_cap == 0 or advice.get(fid) == "random":
            _check((ws, wn) == (p, 1), f"readahead off but miss at {p} got window {(ws, wn)}")
            checked_exact += 1
            continue
        st = state.setdefault(fid, {"clock": 0, "recent": [], "streams": [[False, 0, 0, 0] for _ in range(streams)]})
        st["clock"] += 1
        want_near = sum(1 for r in st["recent"] if abs(r - p) <= NEAR_PAGES)
        _check(near == want_near, f"miss at {p}: near count {near}, model {want_near}")
        st["recent"].append(p)
        if len(st["recent"]) > RECENT:
            st["recent"].pop(0)
        slots = st["streams"]
        zone = next((i for i, s in enumerate(slots) if s[0] and s[1] <= p < s[1] + s[2]), None)
        if zone is not None:
            s = slots[zone]
            exp_ws, exp_wn = s[1], min(2 * s[2], ra_cap)
            slots[zone] = [True, exp_ws + exp_wn, exp_wn, st["clock"]]
            _check((ws, wn) == (exp_ws, min(exp_wn, npages - exp_ws)),
                   f"zone decision at {p}: trace {(ws, wn)}, model {(exp_ws, exp_wn)}")
            checked_exact += 1
            continue
        victim = next((i for i, s in enumerate(slots) if not s[0]), None)
        if victim is None:
            victim = min(range(len(slots)), key=lambda i: (slots[i][3], i))
        if want_near >= NEAR_MIN:
            exp_wn = ra_cap
            exp_ws = p - p % ra_cap
            _check((ws, wn) == (exp_ws, min(exp_wn, npages - exp_ws)),
                   f"aggregate decision at {p}: trace {(ws, wn)}, model {(exp_ws, exp_wn)}")
            checked_exact += 1
            slots[victim] = [True, exp_ws + exp_wn, exp_wn, st["clock"]]
        else:
            w0 = ra_init if (p == 0 or advice.get(fid) == "sequential") else 1
            _check(ws == p, f"context decision at {p} starts at {ws}")
            full = wn if p + wn < npages else None        # EOF-clamped windows cannot be classified
            if full is not None:
                _check(full in (1, min(w0, ra_cap)) or (full % 2 == 0 and full <= ra_cap) or full == ra_cap,
                       f"context decision at {p}: window {wn} is not 1, W0 or 2h <= cap")
            checked_shape += 1
            # the device stored the unclamped length; recover it where the window was clamped
            stored = wn if full is not None else max(wn, 1)
            slots[victim] = [True, ws + stored, stored, st["clock"]]
    return {"exact": checked_exact, "shape_only": checked_shape}


def replay_requests(events) -> int:
    """Per block: miss -> its allocations -> one request covering their contiguous run."""
    per_block = defaultdict(list)
    for e in events:
        if e[0] == "MISS":
            per_block[e[1]].append(e)
        elif e[0] == "ALLOC":
            per_block[e[1]].append(e)
        elif e[0] in ("REQ", "NOFRAME"):
            per_block[e[1]].append(e)
    n = 0
    for blk, seq in per_block.items():
        cur = None
        allocs: List[tuple] = []
        for e in seq:
            if e[0] == "MISS":
                # a miss that got no frame at all is retried: it leaves no allocation behind
                _check(cur is None or not allocs, f"block {blk}: miss at {e[3]} before the previous request")
                cur = e
                allocs = []
            elif e[0] == "ALLOC":
                _check(cur is not None, f"block {blk}: allocation outside a miss")
                allocs.append((e[6], e[3]))
            elif e[0] == "REQ":
                _check(cur is not None, f"block {blk}: request without a miss")
                _, _b, fid, p, ws, wn, _near = cur
                # the lanes of one wave append their records in no fixed order; the hand
                # tickets fix the order in which the run's pages were given frames
                pages = [q for _, q in sorted(allocs)]
                _check(pages and pages[0] == p, f"block {blk}: first allocation is not the demanded page {p}")
                lo, hi = min(pages), max(pages)
                _check(sorted(pages) == list(range(lo, hi + 1)), f"block {blk}: request run has holes {sorted(pages)}")
                _check(ws <= lo and hi < ws + wn, f"block {blk}: run {lo}..{hi} outside window {(ws, wn)}")
                _check((e[3], e[4]) == (lo, hi - lo + 1), f"block {blk}: request {e[3:]} != run {(lo, hi - lo + 1)}")
                n += 1
                cur = None
        _check(cur is None or not allocs, f"block {blk}: trailing miss without request")
    return n
