"""MI355X-native D2Q37 thermal lattice Boltzmann hot path.

The compute path is the HIP library `libd2q37.so` (C-ABI, `include/lbm.h`);
`paper_1703_00185_amd.lbm` is its thin ctypes binding.  Importing this
package loads nothing; the library is loaded on first use of the binding.
"""
__all__ = ["lbm", "inputs"]
