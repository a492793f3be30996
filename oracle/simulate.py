"""The three-step lensed-image simulation (oracle, FP64).

Steps in the paper's order (image-simulation section): image-plane grid ->
source-plane positions after all deflections -> source light there (plus the
unlensed lens light) -> supersample average -> PSF convolution.
Reading: supersampled sub-pixels are averaged to native pixels before the
native-resolution PSF is applied.
"""
import numpy as np

from .conv import convolve_same
from .grid import subpixel_coords, supersample_reduce
from .lens import ray_shoot
from .light import surface_brightness


def simulate_unconvolved(scene):
    """Native-pixel lensed image (flux per pixel) before the PSF, (ny, nx)."""
    g = scene.grid
    tx, ty = subpixel_coords(g.nx, g.ny, g.pixel_scale, g.x0, g.y0, g.supersample)
    bx, by = ray_shoot(tx, ty, scene.lens)
    sb = surface_brightness(tx, ty, bx, by, scene.source, scene.lens_light, scene.bn_exact)
    return supersample_reduce(sb, g.pixel_scale)


def simulate_image(scene):
    """Full simulated image (ny, nx): the unconvolved image convolved with the
    scene's PSF (no convolution when the scene has none)."""
    img = simulate_unconvolved(scene)
    if scene.psf is None:
        return img
    return convolve_same(img, scene.psf)
