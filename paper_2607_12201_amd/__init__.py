"""MI355X-native interior-point Newton step for Radau collocation of ODE parameter estimation.

The computation lives in libcolloc.so (hand-written HIP for gfx950, C ABI in include/colloc.h);
``paper_2607_12201_amd.colloc`` is its ctypes binding and ``workloads`` the seeded synthetic
problem generator.  Importing the package does not load the library.
"""
