"""MI355X-native fast matching pursuit on multi-Gabor dictionaries.

The compute path lives in the HIP library ``libmpg.so`` (C-ABI declared in
``include/mpg.h``); ``paper_2202_12380_amd.mpg`` is its thin ctypes binding.
Importing this package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
