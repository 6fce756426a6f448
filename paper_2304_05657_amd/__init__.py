"""MI355X-native coupled lattice-Boltzmann / finite-difference step for
low-Mach reacting flow in porous media (Hosseini & Thevenin,
arXiv:2304.05657).

The step runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/lbfd.h`` (``liblbfd.so``); :mod:`.lbfd` is the thin
ctypes binding and :mod:`.workloads` builds the seeded synthetic inputs.
"""
__all__ = ["lbfd", "workloads"]
