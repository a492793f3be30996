"""Error metrics shared by the GPU parity tests.

Deflections: e_alpha = max_i |alpha_gpu,i - alpha_orc,i|_2 /
                       max(|alpha_orc,i|_2, 1e-3 max_j |alpha_orc,j|_2)   (bar 1e-5)
Images:      e_I     = max_i |I_gpu,i - I_orc,i| /
                       max(|I_orc,i|, 1e-3 max_j |I_orc,j|)                 (bar 1e-4)
The floor keeps FP32 underflow of far light tails and round-off in faint pixels
from dominating a pure relative error.
"""
import numpy as np

DEFLECTION_TOL = 1e-5
IMAGE_TOL = 1e-4


def deflection_error(ax, ay, ex, ey):
    ax, ay = np.asarray(ax, np.float64), np.asarray(ay, np.float64)
    ex, ey = np.asarray(ex, np.float64), np.asarray(ey, np.float64)
    ref = np.hypot(ex, ey)
    den = np.maximum(ref, 1e-3 * ref.max()) if ref.size else ref
    return float(np.max(np.hypot(ax - ex, ay - ey) / den)) if ref.size else 0.0


def image_error(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    if ref.size == 0:
        return 0.0
    scale = np.abs(ref).max()
    if scale == 0.0:
        return float(np.abs(got).max())
    den = np.maximum(np.abs(ref), 1e-3 * scale)
    return float(np.max(np.abs(got - ref) / den))
