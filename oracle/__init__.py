"""CPU oracle for the GPU file page cache -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run anything in this package. The product path (the
HIP library and its Python binding) never calls it, and this package shares no
code with that path; both read the same synthetic inputs from ``workloads``.

Modules:

* ``data``   -- what gread() must deliver: plain ``pread`` of the file, and the
  per-block checksums / histograms of the benchmark consumers, from their plain
  definitions.
* ``policy`` -- a step-by-step model of the page-cache, readahead and clock
  replacement policy (the paper's GPU-side prefetch mechanism and replacement,
  with the readings listed in the design notes), run either in a serialized
  order (predicts the whole trace) or replayed on a recorded trace.
* ``naive``  -- a second, independently written policy model (plain lists,
  linear scans) used only to cross-check ``policy`` by brute force.
* ``lra``    -- the paper's per-threadblock least-recently-allocated replacement,
  used as a pin on the eviction order of read-once streams.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
(published SplitMix64 vector, closed forms, brute force on tiny inputs,
invariants, the paper's worked readahead example); none is "parity unpinned".
"""
