"""MI355X-native shaped-EOS pseudopotential lattice Boltzmann hot path (HIP, gfx950).

The method runs in liblbm.so (include/lbm.h); ``lbm`` is its thin ctypes binding.
"""
from . import lbm  # noqa: F401
