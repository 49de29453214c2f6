"""MI355X-native FDTD hot path of the elecode method (Kuklin, arXiv 2207.06908).

The Yee leapfrog update of E and H with lossy coefficients, a thin-wire
sub-cell model, lumped current sources and a convolutional PML runs as
hand-written HIP kernels for gfx950 behind a C-ABI library
(``include/fdtd.h``).  ``paper_2207_06908_amd.fdtd`` is the Python binding;
``paper_2207_06908_amd.scenarios`` builds the seeded synthetic workloads.
"""
