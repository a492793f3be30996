"""MI355X-native lensed-image simulation (JAXtronomy's three-step pipeline).

The compute path is libjt.so: hand-written HIP kernels for gfx950 behind the C
ABI of include/jt.h.  This package is its thin Python binding; `Context`
exposes the same calls as the ABI (ray_shoot, deflection, source_sb,
convolve, simulate_image, upload_subhalos, upload_psf, ...) on torch CUDA
tensors and torch's current HIP stream.
"""
from ._native import (Context, JtError, LIB_PATH, Server, convolve_auto_method, load_library, pso_move,
                      sersic_bn, uniform, STATUS_NAMES)

__all__ = ["Context", "JtError", "LIB_PATH", "Server", "convolve_auto_method", "load_library", "pso_move",
           "sersic_bn", "uniform", "STATUS_NAMES"]
