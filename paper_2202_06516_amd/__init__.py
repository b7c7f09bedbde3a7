"""MI355X-native multiphase lattice Boltzmann step with in-step contact-angle measurement.

The compute path is liblbm.so (hand-written HIP for gfx950, C ABI in
include/lbm.h); ``lbm`` is its ctypes binding, ``workloads`` the seeded
synthetic inputs.  Build with ``python -m paper_2202_06516_amd.build``.
"""
