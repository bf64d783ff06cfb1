"""MI355X-native dynamical perturbation theory (arXiv:2002.12872).

The compute path is the HIP library ``_lib/libdpt.so`` (C ABI in
``include/dpt.h``); ``paper_2002_12872_amd.dpt`` is its ctypes binding and
``paper_2002_12872_amd.build`` compiles it for gfx950.  Nothing is imported
eagerly here, so importing the package never touches the GPU.
"""
