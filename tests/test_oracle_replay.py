"""The concurrent-trace replay checker (oracle.replay), pinned on the CPU.

It must accept traces that follow the rules -- here the serialized model's own traces,
re-labelled with tickets and blocks -- and reject traces with a planted mistake: a wrong
eviction victim, a page held twice, a reused ticket, a wrong window, a request with a hole.
"""
import random

import pytest

from oracle import replay
from oracle.policy import PolicyModel, run_serialized
from workloads import configs


def _to_replay(model):
    """Model events -> replay tuples: give ALLOC the ticket of the claim before it and the
    block of the current miss; give HAND the block too; pack each miss's detector inputs
    (near | h << 8 | rule << 24) the way the device trace does."""
    out = []
    blk = -1
    last_claim = None
    decisions = iter(model.decisions)
    for e in model.events:
        if e[0] == "MISS":
            blk = e[1]
            near, h, rule = next(decisions)
            out.append(("MISS", blk, e[2], e[3], e[4], e[5], near | h << 8 | rule << 24))
        elif e[0] == "HAND":
            out.append(("HAND",) + tuple(e[1:]) + (blk,))
            if e[3] in ("FREE", "EVICT"):
                last_claim = e[1]
        elif e[0] == "ALLOC":
            out.append(("ALLOC", blk, e[1], e[2], e[3], e[4], last_claim))
        elif e[0] == "REQ":
            out.append(("REQ", blk, e[1], e[2], e[3]))
        elif e[0] == "NOFRAME":
            out.append(e)
    return out


def _model_trace(name, cap, recent=64, near_pages=64, near_min=3):
    wl = configs.get(name)
    C = wl.cache_bytes // wl.page_size
    m = PolicyModel(C, wl.page_size, ra_init_pages=4, ra_cap_pages=cap, streams_per_file=8, recent=recent,
                    near_pages=near_pages, near_min=near_min)
    m.open(0, wl.file.size)
    run_serialized(m, 0, wl.offsets, wl.read_size)
    ev = _to_replay(m)
    return wl, C, m, ev


@pytest.mark.parametrize("name,cap,det", [("c2_small", 0, (64, 64, 3)), ("c2_small", 16, (64, 64, 3)),
                                          ("c3c_small", 8, (64, 64, 3)), ("c3a_small", 16, (64, 64, 3)),
                                          ("c2_small", 16, (8, 4, 2)), ("c3b_small", 8, (16, 8, 2)),
                                          ("c3a_small", 8, (64, 64, 65)), ("c3c_small", 8, (64, 64, 65))])
def test_replay_accepts_rule_following_traces(name, cap, det):
    wl, C, m, ev = _model_trace(name, cap, *det)
    rc = replay.replay_clock(ev, C)
    assert [(f, p) for _, _, f, p in rc["evictions"]] == \
        [(e[4], e[5]) for e in m.events if e[0] == "HAND" and e[3] == "EVICT"]
    assert rc["allocations"] == m.fetched_pages and rc["wasted_pages"] == m.wasted_pages
    rr = replay.replay_readahead(ev, 4, cap, 8, {0: wl.file.size}, wl.page_size, recent=det[0],
                                 near_pages=det[1], near_min=det[2])
    assert rr["exact"] == m.misses and rr["shape_only"] == 0
    assert replay.replay_requests(ev) == m.requests


def test_replay_rejects_hand_action_against_what_it_found():
    """Each visit's action must follow from the bits it read: a CLEAR of a frame whose bit
    was clear, an EVICT of a frame whose bit was set or that was pinned, a SKIP of a free,
    unpinned frame without a lost race -- each is rejected."""
    wl, C, m, ev = _model_trace("c2_small", 16)
    for act, tweak in (("CLEAR", lambda s: s & ~1), ("EVICT", lambda s: s | 1), ("EVICT", lambda s: s | 2),
                       ("SKIP", lambda s: 0), ("FREE", lambda s: s | 3 << 3)):
        if not any(e[0] == "HAND" and e[3] == act for e in ev):
            continue
        bad = _mutate(ev, lambda e: e[0] == "HAND" and e[3] == act, lambda e: e[:7] + (tweak(e[7]),) + e[8:])
        with pytest.raises(replay.ReplayError):
            replay.replay_clock(bad, C)


def test_replay_rejects_context_window_not_sized_by_history():
    """A context decision's window is min(2h, cap) for the history h the trace reports."""
    wl, C, m, ev = _model_trace("c3a_small", 8, near_min=65)     # aggregate rule off
    ctx = [e for e in ev if e[0] == "MISS" and (e[6] >> 24) == 3]
    assert ctx, "no context decision in the model trace"
    assert replay.replay_readahead(ev, 4, 8, 8, {0: wl.file.size}, wl.page_size, near_min=65)["by_rule"][3] == len(ctx)
    bad = _mutate(ev, lambda e: e is ctx[0], lambda e: e[:6] + (e[6] + (1 << 8),))
    with pytest.raises(replay.ReplayError):
        replay.replay_readahead(bad, 4, 8, 8, {0: wl.file.size}, wl.page_size, near_min=65)


def _mutate(ev, pred, fn):
    out = list(ev)
    for i, e in enumerate(out):
        if pred(e):
            out[i] = fn(e)
            return out
    raise AssertionError("nothing to mutate")


def test_replay_rejects_wrong_victim():
    wl, C, m, ev = _model_trace("c2_small", 0)
    bad = _mutate(ev, lambda e: e[0] == "HAND" and e[3] == "EVICT", lambda e: e[:5] + (e[5] + 1,) + e[6:])
    with pytest.raises(replay.ReplayError):
        replay.replay_clock(bad, C)


def test_replay_rejects_page_held_twice():
    wl, C, m, ev = _model_trace("c2_small", 0)
    allocs = [e for e in ev if e[0] == "ALLOC"]
    # allocate the first page again at the second claim while it is still resident
    first = allocs[0]
    bad = _mutate(ev, lambda e: e is allocs[1], lambda e: e[:2] + (first[2], first[3]) + e[4:])
    with pytest.raises(replay.ReplayError):
        replay.replay_clock(bad, C)


def test_replay_rejects_reused_ticket():
    wl, C, m, ev = _model_trace("c2_small", 0)
    hands = [e for e in ev if e[0] == "HAND"]
    bad = _mutate(ev, lambda e: e is hands[5], lambda e: (e[0], hands[4][1]) + e[2:])
    with pytest.raises(replay.ReplayError):
        replay.replay_clock(bad, C)


def test_replay_rejects_wrong_window():
    wl, C, m, ev = _model_trace("c2_small", 16)
    misses = [e for e in ev if e[0] == "MISS"]
    target = misses[3]
    bad = _mutate(ev, lambda e: e is target, lambda e: e[:5] + (e[5] + 1,) + e[6:])
    with pytest.raises(replay.ReplayError):
        replay.replay_readahead(bad, 4, 16, 8, {0: wl.file.size}, wl.page_size)


def test_replay_rejects_request_with_hole():
    wl, C, m, ev = _model_trace("c2_small", 16)
    reqs = [e for e in ev if e[0] == "REQ" and e[4] >= 3]
    bad = _mutate(ev, lambda e: e is reqs[0], lambda e: e[:4] + (e[4] + 1,))
    with pytest.raises(replay.ReplayError):
        replay.replay_requests(bad)


def test_replay_requests_orders_allocations_by_ticket():
    """Records of one wave's allocations may appear in any order; the tickets decide. Swapping
    two records keeps the trace valid; giving the demanded page a later ticket does not."""
    wl, C, m, ev = _model_trace("c2_small", 16)
    n = replay.replay_requests(ev)
    # the first two allocations of one request (same block, no MISS or REQ between them)
    i = j = None
    for k, e in enumerate(ev):
        if e[0] == "MISS":
            i = None
        elif e[0] == "ALLOC":
            if i is None:
                i = k
            elif ev[i][1] == e[1]:
                j = k
                break
    assert i is not None and j is not None
    swapped = list(ev)
    swapped[i], swapped[j] = ev[j], ev[i]
    assert replay.replay_requests(swapped) == n
    a, b = ev[i], ev[j]
    retick = list(ev)
    retick[i] = a[:6] + (b[6],)
    retick[j] = b[:6] + (a[6],)
    with pytest.raises(replay.ReplayError):
        replay.replay_requests(retick)
