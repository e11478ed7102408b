"""MI355X-native (gfx950) N-phase conservative Allen-Cahn + Navier-Stokes lattice
Boltzmann step: hand-written HIP kernels behind a C ABI (libnphase_lbm.so), with a thin
Python binding.  The binding is imported lazily so that `inputs` stays dependency-free."""

__all__ = ["inputs", "binding"]
