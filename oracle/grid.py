"""Image-plane coordinate grid and supersampling (oracle, FP64).

The first step of the paper's image simulation (image-simulation section)
starts from a grid of image-plane angles.  The paper does not fix its
convention; the reading used here: pixel (i, j) has row i along +y and column j along +x, the
grid is centred on (x0, y0), and each pixel is split into s x s equal
sub-pixels evaluated at their centres.  A native pixel value is the mean of its
sub-pixel surface brightness times the pixel area (flux per pixel).
"""
import numpy as np


def subpixel_coords(nx, ny, pixel_scale, x0=0.0, y0=0.0, s=1):
    """Sub-pixel centre angles.

    Returns (tx, ty), float64 arrays of shape (ny, nx, s, s) indexed
    [row i, column j, sub-row a, sub-column b], with
      tx = x0 + (j - (nx-1)/2) * d + ((b + 1/2)/s - 1/2) * d
      ty = y0 + (i - (ny-1)/2) * d + ((a + 1/2)/s - 1/2) * d.
    """
    d = float(pixel_scale)
    j = np.arange(nx, dtype=np.float64)[None, :, None, None]
    i = np.arange(ny, dtype=np.float64)[:, None, None, None]
    b = np.arange(s, dtype=np.float64)[None, None, None, :]
    a = np.arange(s, dtype=np.float64)[None, None, :, None]
    tx = x0 + (j - (nx - 1) / 2.0) * d + ((b + 0.5) / s - 0.5) * d
    ty = y0 + (i - (ny - 1) / 2.0) * d + ((a + 0.5) / s - 0.5) * d
    shape = (ny, nx, s, s)
    return np.broadcast_to(tx, shape).copy(), np.broadcast_to(ty, shape).copy()


def supersample_reduce(sb, pixel_scale):
    """Pixel value = pixel area x mean of the s x s sub-pixel surface
    brightness.  `sb` has shape (ny, nx, s, s); returns (ny, nx)."""
    sb = np.asarray(sb, dtype=np.float64)
    return float(pixel_scale) ** 2 * sb.mean(axis=(2, 3))
