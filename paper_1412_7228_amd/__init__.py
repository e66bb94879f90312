"""MI355X-native pseudo-potential MRT lattice Boltzmann with tunable surface tension.

The update (density/psi pass, Kupershtokh force, MRT collision with the force
source and the pressure-tensor term, streaming) runs in hand-written HIP
kernels for gfx950 inside ``liblbm.so``; :mod:`.lbm` is the ctypes binding of
its C ABI (``include/lbm.h``).  Importing the package loads nothing.
"""
__all__ = ["inputs"]
