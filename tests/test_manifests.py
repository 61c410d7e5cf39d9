"""Pins for the frozen multi-file manifests (CPU only): the files under workloads/manifests
are what the generator writes, sizes follow the stated lognormal recipe and clips, arrivals
are a Poisson stream of the stated rate with uniformly chosen files, and the admission
checker of the serving oracle rejects planted violations."""
import math

import numpy as np
import pytest

from oracle import serve as oserve
from workloads import manifest, splitmix

MiB, GiB = 1 << 20, 1 << 30


@pytest.mark.parametrize("name,builder", [("batch", lambda: manifest.build_batch(False)),
                                          ("batch_small", lambda: manifest.build_batch(True)),
                                          ("serve", lambda: manifest.build_serve(False)),
                                          ("serve_small", lambda: manifest.build_serve(True))])
def test_frozen_files_match_generator(name, builder):
    assert manifest.load(name) == builder()


def test_uniforms_are_top_53_bits():
    x = splitmix.output_int(1000005, 1)
    assert manifest._uniforms(1000005, 1)[0] == (x >> 11) / 2.0 ** 53


def test_normals_moments():
    z = np.array(manifest.normals(1000005, 4000))
    assert abs(z.mean()) < 0.06 and abs(z.std() - 1.0) < 0.05
    # the Box-Muller cosine branch has the normal's symmetric tails
    assert 0.040 < np.mean(z > 1.645) < 0.062 and 0.040 < np.mean(z < -1.645) < 0.062


def test_serve_pool_is_prefix_of_full_pool_and_clipped():
    m = manifest.load("serve")
    full = manifest.lognormal_sizes(1000005, 512, 128 * MiB, 1.2, 16 * MiB, 4 * GiB)
    sizes = [f["size"] for f in m["files"]]
    assert sizes == full[:64]
    assert all(16 * MiB - 8 < s <= 4 * GiB and s % 8 == 0 for s in full)
    # median of the lognormal is 128 MiB: about half the full pool lies below it
    assert 0.4 < np.mean(np.array(full) < 128 * MiB) < 0.6
    assert m["budget_bytes"] == sum(sizes) // 4 // GiB * GiB
    assert [f["seed"] for f in m["files"]] == [10000 + j for j in range(64)]


@pytest.mark.parametrize("name", ["serve", "serve_small"])
def test_arrivals_are_poisson_with_uniform_files(name):
    m = manifest.load(name)
    rate = m["rate_per_s"]
    t = np.array([r["t_ns"] for r in m["requests"]], dtype=np.float64)
    f = np.array([r["file"] for r in m["requests"]])
    gaps = np.diff(np.concatenate([[0.0], t])) / 1e9
    assert np.all(gaps >= 0)
    n = len(gaps)
    # mean gap 1/rate within 4 standard errors; exponential: P(gap > mean) = 1/e
    assert abs(gaps.mean() * rate - 1.0) < 4.0 / math.sqrt(n)
    assert abs(np.mean(gaps * rate > 1.0) - math.exp(-1.0)) < 4.0 * math.sqrt(0.25 / n)
    pool = len(m["files"])
    assert f.min() >= 0 and f.max() < pool
    counts = np.bincount(f, minlength=pool)
    chi2 = float(((counts - n / pool) ** 2 / (n / pool)).sum())
    assert chi2 < pool + 6 * math.sqrt(2 * pool)


def test_scaled_arrivals():
    m = manifest.load("serve")
    base = [r["t_ns"] for r in m["requests"]]
    assert manifest.scaled_arrivals(m, 200) == base
    assert manifest.scaled_arrivals(m, 50) == [t * 4 for t in base]


def _records(admit, done, reserved):
    n = len(admit)
    return dict(arrival_ns=[0] * n, admit_ns=admit, done_ns=done, seq=list(range(n)), reserved=reserved)


def test_admission_checker_accepts_and_rejects():
    ok = _records(admit=[0, 1, 5, 10], done=[4, 9, 8, 12], reserved=[4, 4, 4, 8])
    assert oserve.check_admission(budget=8, **ok) == 8
    # planted: the second request pushes the total to 12 while the first is in flight
    bad = _records(admit=[0, 1, 5, 6], done=[4, 9, 8, 10], reserved=[4, 8, 4, 8])
    with pytest.raises(oserve.AdmissionError):
        oserve.check_admission(budget=8, **bad)
    # a request larger than the budget is fine when it runs alone
    alone = _records(admit=[0, 5], done=[4, 9], reserved=[20, 4])
    assert oserve.check_admission(budget=8, **alone) == 20
    # planted: admitted out of arrival order
    swapped = _records(admit=[0, 1], done=[2, 3], reserved=[1, 1])
    swapped["seq"] = [1, 0]
    with pytest.raises(oserve.AdmissionError):
        oserve.check_admission(budget=8, **swapped)
    # planted: completion before admission
    early = _records(admit=[0, 5], done=[4, 3], reserved=[1, 1])
    with pytest.raises(oserve.AdmissionError):
        oserve.check_admission(budget=8, **early)


def test_reservation_rounds_to_pages():
    assert oserve.reservation(0, 4096) == 0
    assert oserve.reservation(1, 4096) == 4096
    assert oserve.reservation(8192, 4096) == 8192


def test_readpeak_reads_every_byte(tmp_path):
    """The storage-rate timer reads each file whole (or up to the limit), across threads."""
    from workloads import configs
    a = tmp_path / "a.bin"
    b = tmp_path / "b.bin"
    a.write_bytes(bytes(range(256)) * 4096 * 3 + b"x" * 123)     # not a multiple of the chunk
    b.write_bytes(b"\0" * (1 << 20))
    exe = configs.build_readpeak()
    import subprocess
    out = subprocess.check_output([exe, "3", str(256 << 10), "0", str(a), str(b)], text=True).split()
    assert int(out[0]) == a.stat().st_size + b.stat().st_size and float(out[1]) > 0
    out = subprocess.check_output([exe, "2", str(64 << 10), str(512 << 10), str(a)], text=True).split()
    assert int(out[0]) == 512 << 10
    assert configs.read_peak([str(a), str(b)], threads=2, chunk=64 << 10) > 0
