"""MI355X-native nonlocal potentials of the NLSE via the NUFFT (Bao, Jiang, Tang, Zhang).

The compute path is the C-ABI library libnlf.so (include/nlf.h), built from csrc/ for
gfx950.  `paper_1410_3584_amd.nlf` is a thin ctypes binding with the same names; it only
marshals arguments (torch tensors are used for device memory and streams).  Importing this
package does not load the library; `nlf.load()` does, and raises if it is missing.
"""
__all__ = ["nlf", "inputs"]
