"""Suffix-array matching of short DNA reads on the AMD MI355X (gfx950).

The compute path is the HIP library libsamatch.so (see include/samatch.h);
this package holds its sources (csrc/), its build script and a ctypes
binding with the same names as the C-ABI.
"""
from .samatch import *  # noqa: F401,F403
from . import samatch  # noqa: F401
