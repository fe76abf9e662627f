"""MI355X-native M-HDC SpMV (arXiv:2105.04937).

The compute path lives in the HIP library ``libmhdc.so`` (C-ABI declared in
``include/mhdc.h``); ``paper_2105_04937_amd.mhdc`` is its thin ctypes binding.
``paper_2105_04937_amd.synth`` draws the seeded synthetic inputs.
Importing this package loads nothing; the binding loads the library on first
use and raises if it has not been built.
"""
