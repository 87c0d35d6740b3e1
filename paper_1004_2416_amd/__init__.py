"""MI355X-native (gfx950, HIP) implementation of the coupled immersed
boundary / lattice Boltzmann / finite element capsule timestep of Krueger,
Varnik and Raabe (arXiv:1004.2416).

The compute path lives in the C-ABI shared library built from csrc/ (declared
in include/ibm_lbm.h); `binding` is its thin ctypes binding, which uses
PyTorch only for device memory and streams.  Importing this package does not
load the library; `from paper_1004_2416_amd import binding` does, and fails
loudly if it has not been built.
"""
__all__ = ["binding", "workloads"]
