"""What the serving loop must produce, and the admission rule its records must obey.

Test infrastructure only (see the package docstring).

* Each request reads one whole file, so its checksum is the file's checksum (wrapping u64
  sum of little-endian u32 words, trailing partial word zero-padded) and its result is the
  file size, whatever else runs beside it.
* Admission (the serving design's rule, built on the cache budget): requests are admitted in
  arrival order; when request r is admitted, the reservations of admitted requests the host
  has not yet seen complete, plus r's own, stay within the budget, unless nothing else is in
  flight. A reservation is the file size rounded up to whole pages.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


class AdmissionError(AssertionError):
    pass


def reservation(size: int, page_size: int) -> int:
    return -(-size // page_size) * page_size


def check_admission(arrival_ns: Sequence[int], admit_ns: Sequence[int], done_ns: Sequence[int],
                    seq: Sequence[int], reserved: Sequence[int], budget: int) -> int:
    """Check FIFO order and the budget at every admission; returns the largest in-flight
    reservation total seen. Records are in request (arrival) order."""
    arrival = np.asarray(arrival_ns, dtype=np.int64)
    admit = np.asarray(admit_ns, dtype=np.int64)
    done = np.asarray(done_ns, dtype=np.int64)
    order = np.asarray(seq, dtype=np.int64)
    res = np.asarray(reserved, dtype=np.int64)
    n = len(arrival)
    if sorted(order.tolist()) != list(range(n)):
        raise AdmissionError("admission numbers are not a permutation")
    if np.any(np.diff(order) != 1) and n > 1:
        raise AdmissionError("requests were not admitted in arrival order")
    if np.any(admit < arrival):
        raise AdmissionError("a request was admitted before it arrived")
    if np.any(done < admit):
        raise AdmissionError("a request completed before it was admitted")
    peak = 0
    for r in range(n):
        inflight = [q for q in range(n) if order[q] < order[r] and done[q] > admit[r]]
        total = int(res[inflight].sum()) + int(res[r])
        if inflight and total > budget:
            raise AdmissionError(f"request {r} admitted with {total} bytes reserved > budget {budget}")
        peak = max(peak, total)
    return peak
