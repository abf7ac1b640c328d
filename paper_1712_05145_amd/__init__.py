"""MI355X (gfx950) FFT-based homogenization of orders 0 and 1 (arXiv:1712.05145).

The compute path is libffth.so (HIP kernels behind the C-ABI in
include/ffth.h); ``ffth`` is its ctypes binding and ``microstructure`` holds
the seeded synthetic inputs.
"""
