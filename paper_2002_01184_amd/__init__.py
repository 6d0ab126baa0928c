"""MI355X-native batched Hamiltonian Monte Carlo (arXiv 2002.01184, Sec. 2.1).

The sampler runs in hand-written HIP kernels for gfx950 behind the C ABI in
include/hmc.h (libhmc.so).  `paper_2002_01184_amd.hmc` is the thin ctypes
binding with the same entry-point names; `diagnostics` holds host-side
R-hat / ESS for measurement.  Importing this package does not load the GPU
library; the binding loads it on first use and raises if it is missing.
"""
__all__ = ["hmc", "diagnostics"]
