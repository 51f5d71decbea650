"""MI355X-native coupled pseudopotential / improved-thermal lattice Boltzmann.

The product is the C-ABI library ``liblbpc.so`` (hand-written HIP kernels for
gfx950) declared in ``include/lbpc.h``; :mod:`paper_1709_04400_amd.lbpc` is its
ctypes binding.  :mod:`paper_1709_04400_amd.inputs` holds the seeded input
generators (parameters and initial fields, no arithmetic of the method).
Importing the package loads nothing native; the binding loads the library on
first use and raises if it is missing.
"""
__all__ = ["lbpc", "inputs"]
