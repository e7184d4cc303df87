"""MI355X (gfx950) implementation of the time step of the two-population
Particles-on-Demand kinetic model of compressible multiphase flow (Reyhanian,
Dorschner & Karlin, arXiv:2002.09217).

    paper_2002_09217_amd.pond       binding of the C ABI (include/pond.h)
    paper_2002_09217_amd.workloads  seeded synthetic inputs shaped like the paper's cases
    paper_2002_09217_amd.build      hipcc build of libpond.so

Importing the package loads nothing; ``pond.load()`` loads the library.
"""
