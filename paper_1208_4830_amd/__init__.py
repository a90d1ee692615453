"""libsblm: MI355X-native batched fitness evaluation and evolutionary fitting
of static binary-lens microlensing lightcurves (Rajpaul 2012).

The compute path is the HIP library libsblm.so (C ABI in include/sblm.h);
`paper_1208_4830_amd.sblm` is its thin ctypes binding.  Importing the package
loads nothing; `sblm.load()` does, and raises if the library is missing.
"""
