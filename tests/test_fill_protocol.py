"""The device's page-fill protocol as a CPU thread model, under ThreadSanitizer.

tests/csrc/fill_protocol_model.cpp restates the device's steps on the library's real layout
(frame-word bits, gfs_req_dev, gfs_rpc_slot) with host threads standing in for blocks and one
for the host I/O threads: requesters take frames, post into ring slots whose previous
generation is free, wait for the host, publish the request, claim (PULL bit) and copy the
frames no helper took, publish them and count them off, the last one freeing the slot; joiners
copy their own frames once the request (synchronous) or the ring slot (asynchronous window)
says the bytes are staged; windows take slots of their own without waiting. The frame pool is
small, so requesters wait for frames other readers hold. Every posted frame must be published
once with the right bytes, every slot generation freed in order, no wait may pass its deadline,
and ThreadSanitizer must see no race. Two planted mistakes must be caught by the deadlines:
windows sharing the ticketed slots (the stall seen on the GPU), and a poster that waits for its
slot's completion to equal its own generation after helpers have published the whole window.
The lock-free one-page reservation must leave exactly one entry per key.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("no g++")
    out = str(tmp_path_factory.mktemp("fpm") / "fill_protocol_model")
    subprocess.check_call([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
                           "-I", os.path.join(ROOT, "include"), "-o", out,
                           os.path.join(ROOT, "tests", "csrc", "fill_protocol_model.cpp")])
    return out


def _run(model, args, deadline_s=60):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66", FPM_DEADLINE_S=str(deadline_s))
    return subprocess.run([model] + [str(a) for a in args], capture_output=True, text=True, timeout=300, env=env)


@pytest.mark.parametrize("args", [
    ("sync", 16, 40, 128, 8, 4),     # more blocks than slots
    ("sync", 32, 30, 64, 4, 8),      # frame pressure: 32 requesters of 8 frames share 64
    ("async", 16, 40, 128, 8, 4),    # every other request an asynchronous window
    ("async", 24, 30, 64, 4, 16),    # 16-page windows, one slot of their own
    ("async", 32, 40, 256, 8, 8),
    ("reserve", 8, 200, 0, 1, 1),    # eight blocks reserve one key, 200 rounds
])
def test_protocol_model_holds(model, args):
    r = _run(model, args)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.stdout, r.stderr[-2000:])
    assert r.stdout.strip().endswith("-> ok")


def test_planted_exact_generation_wait_is_caught(model):
    # the poster of an asynchronous window that waits for the slot's completion to equal its
    # request's generation never returns once helpers have published every frame and the slot
    # has gone to a later request (the device accepts any later generation)
    r = _run(model, ("async-exact-gen", 16, 40, 128, 2, 4), deadline_s=5)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 1 and "poster: host deadline" in r.stderr, (r.stdout, r.stderr[-2000:])


def test_planted_shared_window_slots_are_caught(model):
    # asynchronous windows that take ticketed slots of the shared ring: a requester waits for a
    # slot held by a window whose pages lie ahead of every reader, while the window's poster
    # waits on that requester's page
    r = _run(model, ("async-shared-slots", 24, 40, 64, 4, 4), deadline_s=5)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 1 and "slot: deadline" in r.stderr, (r.stdout, r.stderr[-2000:])
