"""MI355X-native overlap-operator hot path (arXiv:1106.4964).

The compute lives in libovl.so (HIP kernels for gfx950 behind the C ABI of
include/ovl.h).  `paper_1106_4964_amd.ovl` is its ctypes binding; `build`
compiles the library in-tree.
"""
