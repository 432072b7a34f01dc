"""MI355X-native MPS time evolution of the ab-initio electronic Hamiltonian (tdmps).

The compute path is the HIP library libtdmps.so (C ABI in include/tdmps.h); `tdmps` is
its ctypes binding.
"""
from . import tdmps  # noqa: F401
