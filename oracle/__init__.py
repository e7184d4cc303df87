"""TEST INFRASTRUCTURE ONLY -- the FP64 CPU oracle of the two-population
Particles-on-Demand step (Reyhanian, Dorschner & Karlin, arXiv:2002.09217).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path.
"""
