"""MI355X-native CTU-GLM step (Mignone et al. 2012, Sec. 3): HIP kernels for
gfx950 behind the C ABI of include/ctu.h, with a ctypes binding.

Submodules: ``ctu`` (binding of libctu.so), ``inputs`` (seeded synthetic
workloads), ``build`` (hipcc build of libctu.so).  Importing the package does
not load the shared library; ``ctu.lib()`` does, and raises when it is missing.
"""
