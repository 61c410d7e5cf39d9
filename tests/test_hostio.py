"""The host half of the request ring (csrc/gfs_hostio.h) on the CPU, under ThreadSanitizer.

tests/csrc/hostio_check.cpp links the library's I/O engine with host threads that stand in
for GPU blocks: they post requests into the real ring slots (release store of the slot's
generation), wait for the completion with a deadline (acquire load of done_seq), check every
staged byte and free the slot, as the device does. Each configuration must serve every
request, deliver the right bytes, count them, report -EBADF for an unregistered file and
short reads at the end of a file, and ThreadSanitizer must report no data race.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("no g++")
    out = str(tmp_path_factory.mktemp("hostio") / "hostio_check")
    subprocess.check_call([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
                           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2109_05366_amd", "csrc"),
                           "-o", out, os.path.join(ROOT, "tests", "csrc", "hostio_check.cpp")])
    return out


@pytest.mark.parametrize("backend,threads,slots,producers,requests,direct,depth,pieces", [
    (0, 4, 8, 16, 150, 1, 1, ()),  # shared ring, more blocks than slots, O_DIRECT where allowed
    (0, 8, 64, 32, 60, 0, 1, ()),  # shared ring, buffered reads
    # whole requests in one piece, cut into 64 KiB shares when threads are idle
    (0, 8, 8, 4, 120, 1, 1, (512, 64)),
    (0, 6, 16, 3, 120, 0, 1, (512, 128)),
    (1, 4, 8, 16, 150, 0, 1, ()),  # the partitioned queue (a block's own slot, one thread per range)
    (1, 2, 2, 8, 60, 1, 1, ()),
    (2, 2, 16, 16, 120, 1, 8, ()), # io_uring: 8 reads in flight per thread, O_DIRECT where allowed
    (2, 4, 64, 32, 60, 0, 4, ()),  # io_uring, buffered reads
    (2, 1, 4, 8, 60, 1, 1, ()),    # io_uring, one thread, one read at a time
])
def test_ring_engine_serves_every_request_without_races(checker, tmp_path, backend, threads, slots, producers,
                                                         requests, direct, depth, pieces):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([checker, str(tmp_path), str(backend), str(threads), str(slots), str(producers),
                        str(requests), str(direct), str(depth)] + [str(x) for x in pieces],
                       capture_output=True, text=True, timeout=300, env=env)
    if r.returncode == 5 and "io_uring unavailable" in r.stdout:
        pytest.skip("the kernel refuses io_uring here")
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.stdout, r.stderr[-2000:])
    assert r.stdout.strip().endswith("-> ok")
    if pieces:
        # requests fit one piece of pieces[0] KiB, yet idle threads cut some into smaller shares
        got = dict(kv.split(" ", 1) for kv in r.stdout.split(" -> ")[0].split(", "))
        assert int(got["pieces"]) > int(got["host_requests"]), r.stdout
