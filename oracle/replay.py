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
  eviction order is the EVICT records sorted by ticket. Each visit also logs what it found
  (frame state, reference bit, pin, a lost compare-and-swap), and the action must be the
  second-chance rule applied to it: FREE only on a free frame, CLEAR only on a valid
  unpinned frame with the bit set, EVICT only on a valid unpinned frame with the bit clear,
  SKIP only on a pinned or filling frame or after losing a race;
* readahead: the misses of a file are logged under its miss lock, so their record order
  is the order the detector saw them. Replaying the stream table and the recent-miss
  ring gives the exact window of every decision, and the exact near count; a decision by
  the context rule depends on which pages were cached at that instant, which the trace
  records (the history length h), so its window is checked exactly given h;
* requests: each block's own records are in program order, so every miss is followed by
  that block's allocations and one request, which must cover exactly the contiguous run
  of allocated pages inside the window, starting with the demanded page.

Events are tuples:
  ("MISS", block, file, page, ws, wn, packed[, req])   packed = near | h << 8 | rule << 24,
        req = pages of the missing read from page on (1 when absent)
  ("HAND", ticket, frame, action, vfile, vpage, vra, seen, block)
        seen = ref | pinned << 1 | lost race << 2 | state << 3 (0 free, 1 claimed, 2 filling,
        3 valid)
  ("ALLOC", block, file, page, frame, ra, ticket)
  ("REQ", block, file, first, npages)
  ("NOFRAME", block, file, page)
"""
from __future__ import annotations

from collections import defaultdict
from typing import Dict, List, Tuple

from .policy import NEAR_MIN, NEAR_PAGES, RECENT, RULE_AGGREGATE, RULE_CONTEXT, RULE_NEW, RULE_OFF, RULE_ZONE


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
        _, t, f, act, vf, vp, vra, seen, _blk = e
        _check(f == t % nframes, f"ticket {t} visited frame {f}, expected {t % nframes}")
        ref, pinned, lost, state = seen & 1, (seen >> 1) & 1, (seen >> 2) & 1, seen >> 3
        # the second-chance rule applied to what the visit found
        if act == "FREE":
            _check(state == 0 and not pinned and not lost, f"FREE at ticket {t} found {seen:#x}")
        elif act == "CLEAR":
            _check(state == 3 and ref and not pinned and not lost, f"CLEAR at ticket {t} found {seen:#x}")
            _check(f in occupant, f"CLEAR at ticket {t} of empty frame {f}")
        elif act == "EVICT":
            _check(state == 3 and not ref and not pinned and not lost, f"EVICT at ticket {t} found {seen:#x}")
        else:
            _check(pinned or lost or state in (1, 2), f"SKIP at ticket {t} found {seen:#x}")
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
                     files: Dict[int, int], page_size: int, advice: Dict[int, str] = None,
                     recent: int = RECENT, near_pages: int = NEAR_PAGES, near_min: int = NEAR_MIN):
    """Replay every file's miss decisions in lock (record) order. ra_cap is the cap after the
    thrash guard. Returns how many decisions were checked exactly, and by which rule."""
    advice = advice or {}
    state = {}
    by_rule = defaultdict(int)
    checked_exact = 0
    for e in events:
        if e[0] != "MISS":
            continue
        blk, fid, p, ws, wn, packed = e[1:7]
        req = e[7] if len(e) > 7 else 1
        near, h, rule = packed & 0xFF, (packed >> 8) & 0xFFFF, packed >> 24
        npages = (files[fid] + page_size - 1) // page_size
        if ra_cap == 0 or advice.get(fid) == "random":
            _check((ws, wn) == (p, 1) and rule == RULE_OFF, f"readahead off but miss at {p} got window {(ws, wn)}")
            checked_exact += 1
            by_rule[RULE_OFF] += 1
            continue
        st = state.setdefault(fid, {"clock": 0, "recent": [], "streams": [[False, 0, 0, 0] for _ in range(streams)]})
        st["clock"] += 1
        want_near = sum(1 for r in st["recent"] if abs(r - p) <= near_pages)
        _check(near == want_near, f"miss at {p}: near count {near}, model {want_near}")
        st["recent"].append(p)
        if len(st["recent"]) > recent:
            st["recent"].pop(0)
        slots = st["streams"]
        zone = next((i for i, s in enumerate(slots) if s[0] and s[1] <= p < s[1] + s[2]), None)
        if zone is not None:
            s = slots[zone]
            exp_ws, exp_wn = s[1], min(2 * s[2], ra_cap)
            slots[zone] = [True, exp_ws + exp_wn, exp_wn, st["clock"]]
            exp_rule, exp_h = RULE_ZONE, 0
        else:
            victim = next((i for i, s in enumerate(slots) if not s[0]), None)
            if victim is None:
                victim = min(range(len(slots)), key=lambda i: (slots[i][3], i))
            if want_near >= near_min:
                exp_wn = ra_cap
                exp_ws = p - p % ra_cap
                exp_rule, exp_h = RULE_AGGREGATE, 0
            else:
                # the cached history behind p is the trace's; it cannot exceed the pages
                # behind p or max(ceil(cap / 2), r + 1) (where the count stops), and it
                # decides the rule and sizes the window
                r = min(req, ra_cap)
                _check(h <= min(p, max((ra_cap + 1) // 2, r + 1)), f"decision at {p}: history {h} out of range")
                exp_h = h
                # the context rule needs more history than the read; either window covers
                # at least the rest of the read that missed
                if h > r:
                    exp_wn, exp_rule = min(max(2 * h, r), ra_cap), RULE_CONTEXT
                else:
                    w0 = ra_init if (p == 0 or advice.get(fid) == "sequential") else 1
                    exp_wn, exp_rule = max(1, min(max(w0, r), ra_cap)), RULE_NEW
                exp_ws = p
            slots[victim] = [True, exp_ws + exp_wn, exp_wn, st["clock"]]
        _check(rule == exp_rule and h == exp_h, f"miss at {p}: rule {rule} h {h}, model rule {exp_rule} h {exp_h}")
        _check((ws, wn) == (exp_ws, min(exp_wn, npages - exp_ws)),
               f"decision at {p} (rule {rule}): trace {(ws, wn)}, model {(exp_ws, exp_wn)}")
        checked_exact += 1
        by_rule[exp_rule] += 1
    return {"exact": checked_exact, "shape_only": 0, "by_rule": dict(by_rule)}


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
                fid, p, ws, wn = cur[2:6]
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
