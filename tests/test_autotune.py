"""The autotuner's search on the CPU: it finds the optimum of known functions over the
discrete grid, never evaluates a configuration twice, and skips invalid ones."""
from paper_2109_05366_amd import autotune


def test_finds_separable_optimum():
    target = (1 << 20, 16 << 20, 8)
    calls = []

    def f(cfg):
        calls.append(cfg)
        return -sum(abs(autotune.PAGE_SIZES.index(cfg[0]) - 2) for _ in [0]) \
            - abs(autotune.RA_CAPS.index(cfg[1]) - 2) - abs(autotune.BLOCKS_PER_FILE.index(cfg[2]) - 3)

    r = autotune.coordinate_descent(f)
    assert r.best == target
    assert len(calls) == len(set(calls))


def test_skips_invalid_windows():
    # 1 MiB cap with 2 MiB pages is not a whole number of pages; 64 MiB with 64 KiB pages is
    # exactly the 1024-page limit and is allowed
    assert not autotune.valid((2 << 20, 1 << 20, 4))
    assert autotune.valid((64 << 10, 64 << 20, 4))
    seen = []
    r = autotune.coordinate_descent(lambda c: seen.append(c) or 1.0, start=(2 << 20, 4 << 20, 1))
    assert all(autotune.valid(c) for c in seen)
    assert r.best_value == 1.0


def test_coupled_optimum_needs_second_pass():
    # best blocks-per-file depends on the page size: a second sweep finds it
    def f(cfg):
        page, cap, bpf = cfg
        return 10.0 if (page == 64 << 10 and bpf == 16) else (5.0 if page == 64 << 10 else 1.0)

    r = autotune.coordinate_descent(f, start=(256 << 10, 16 << 20, 4))
    assert r.best[0] == 64 << 10 and r.best[2] == 16 and r.best_value == 10.0
