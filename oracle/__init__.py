"""FP64 CPU oracle of the accumulated-summation 2-D Gaussian rasteriser (GaussianImage,
Sec. 3.2 and App. A).

TEST INFRASTRUCTURE.  Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import, call, link or execute anything in this package.  The GPU path
never imports it and shares no code with it.

``ref`` is the NumPy statement of the method (the correctness authority); ``cref`` loads the same
functions written again in C with OpenMP (``cpu_ref.c``) for large inputs and host timing.
"""
