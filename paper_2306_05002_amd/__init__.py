"""MI355X-native DG residual of the five-equation two-phase model with
Allen-Cahn interface terms (Tonicello & Ihme, arXiv 2306.05002).

The compute path is ``libdg2p.so`` (hand-written HIP for gfx950 behind a C
ABI, sources in ``csrc/``); ``dg2p`` is its thin ctypes binding and
``workloads`` holds the seeded synthetic inputs.  Importing the package does
not load the library; ``paper_2306_05002_amd.dg2p`` does, and fails loudly
when it is missing.
"""
