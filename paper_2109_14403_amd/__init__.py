"""MI355X-native FFT homogenization of thermomechanical composites.

Modules
-------
hom        ctypes binding of libhom.so (the C ABI of include/hom.h)
workloads  seeded synthetic microstructures, material tables, load histories
build      in-tree build of libhom.so for gfx950
surrogate  MLP surrogate with FFT fallback (binding of the surrogate kernels)

Importing the package loads nothing; ``hom.library()`` loads the HIP library
and raises if it is missing.
"""
