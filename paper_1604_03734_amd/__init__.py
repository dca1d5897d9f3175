"""MI355X (gfx950) sparse TSDF fusion and Omega-masked TV primal-dual
regularisation in hashed 8^3 voxel blocks ("DENSER Cities").

The computation lives in libdenser.so (HIP kernels behind the C ABI of
include/denser.h); `denser` is its ctypes binding.
"""
from . import denser  # noqa: F401
