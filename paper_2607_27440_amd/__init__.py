"""MI355X-native kinetic linear stability (kLST) Jacobi-Davidson path.

The compute path lives in the native library ``libklst.so`` (HIP for gfx950,
C-ABI declared in ``include/klst.h``); ``paper_2607_27440_amd.klst`` is its thin
ctypes binding.  ``workloads`` generates seeded synthetic inputs.  Nothing here
is imported eagerly, so the input generator can be used without a GPU.
"""
