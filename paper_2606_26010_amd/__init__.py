"""MI355X-native FAR-LIO registration hot path (voxel hash map + SA-GICP).

The compute lives in the HIP library ``libfar.so`` behind the C ABI declared
in ``include/far.h``; ``paper_2606_26010_amd.far`` is a thin ctypes binding
with the same names.  Importing this package loads nothing; the binding loads
the library on first use and raises if it is missing.
"""
