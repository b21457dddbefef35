"""MI355X (gfx950) GPS L1 C/A acquisition engine -- Python binding.

Thin ctypes layer over ``libgnss_acq.so`` (the C ABI in ``include/gnss_acq.h``).
It only marshals arguments; every step of the search runs in the HIP
kernels of that library.  PyTorch is used only for device memory and streams.
Importing the package raises if the library has not been built: there is no
CPU fallback.
"""
from .binding import *  # noqa: F401,F403
