"""Host logic of the benchmark's HBM-traffic lookup: counted bytes are reported only for
the kernel sources they were taken on, and only under the key asked for."""
import os

import bench


def test_committed_summaries_parse():
    for summary, key in ((bench.TRAFFIC_SUMMARY, "traffic_bytes_per_launch"),
                         (bench.HIT_TRAFFIC_SUMMARY, "traffic_bytes_per_launch_none_1024x16"),
                         (bench.HIT_TRAFFIC_SUMMARY, "traffic_bytes_per_launch_none_512x32"),
                         (bench.HIT_TRAFFIC_SUMMARY, "traffic_bytes_per_launch_none_256x64"),
                         (bench.HIT_TRAFFIC_SUMMARY, "traffic_bytes_per_launch_checksum_512x32")):
        assert os.path.exists(os.path.join(bench.ROOT, summary))
        value, src = bench.recorded_traffic(summary, key)
        if value is None:   # the kernel changed since the counters were taken
            assert src == "kernel changed since the counters were taken"
        else:
            assert src == summary and value > 0


def _write(tmp_path, sha, lines):
    p = tmp_path / "summary.md"
    p.write_text("# counters\n\n" + "".join(f"{k}: {v}\n" for k, v in lines) + f"kernel_source_sha256: {sha}\n")
    return str(p)


def test_current_hash_and_key(tmp_path):
    p = _write(tmp_path, bench.kernel_source_hash(), [("traffic_bytes_per_launch_8x8", "1234  (0.1 GiB)")])
    assert bench.recorded_traffic(p, "traffic_bytes_per_launch_8x8") == (1234, p)
    value, why = bench.recorded_traffic(p, "traffic_bytes_per_launch_9x9")
    assert value is None and "no traffic_bytes_per_launch_9x9" in why


def test_stale_hash_drops_the_figure(tmp_path):
    p = _write(tmp_path, "0" * 64, [("traffic_bytes_per_launch", "1234")])
    assert bench.recorded_traffic(p) == (None, "kernel changed since the counters were taken")


def test_missing_summary(tmp_path):
    assert bench.recorded_traffic(str(tmp_path / "absent.md")) == (None, "no counter summary")
