"""Split-operator solver of the time-dependent Schroedinger equation on one
AMD Instinct MI355X (gfx950): hand-written HIP kernels behind the C ABI of
include/wavepacket.h, with a thin Python binding.

Importing the package loads nothing; `paper_1306_3247_amd.sim` loads the
compiled library and fails loudly when it is missing.
"""
__all__ = ["sim", "workloads", "build"]
