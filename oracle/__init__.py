"""FP64 CPU oracle for the lensed-image simulation -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The HIP library never calls it and shares no
code with it (no kernels, helpers, tables or constants).

What it computes is the paper's three-step image simulation (section
"Improvements over lenstronomy in image simulation"): image-plane angles are
mapped back to the source plane by subtracting every deflector's deflection,
the source light is evaluated at the mapped positions, and the resulting image
is blurred by the PSF.  The paper gives no formulas; every profile below is the standard
closed form from the lensing literature, named in its module, and evaluated in
FP64 with branch forms that are well conditioned.  The direct sum over
deflectors is an exact definition, so the oracle *is* that definition.

Parity pins (closed forms, invariants, quadrature, library routines) live in
tests/test_oracle_*.py.  The input generators are only used as data sources;
the unpinned pieces are listed in `PARITY_UNPINNED`.
"""
from .grid import subpixel_coords, supersample_reduce
from .lens import (sie_deflection, sie_kappa, epl_deflection, epl_kappa, tnfw_G, tnfw_deflection,
                   shear_deflection, nfw_g, nfw_deflection, nfw_kappa, point_mass_deflection, total_deflection,
                   ray_shoot)
from .light import (sersic_bn, sersic, surface_brightness, gaussian, core_sersic, shapelets, shapelet_phi,
                    shapelet_index, component)
from .conv import convolve_at, convolve_same
from .simulate import simulate_image, simulate_unconvolved
from .likelihood import log_likelihood, noise_variance
from .grad import chi2_gradient, macro_vector, macro_names
from .linear import basis_images, linear_amplitudes
from .fit import splitmix64, uniform, pso, pso_start, pso_move, pso_bests, lbfgs

# Functions whose result no independent pin fixes (see the test modules).
PARITY_UNPINNED = ()

__all__ = [
    "subpixel_coords", "supersample_reduce", "sie_deflection", "sie_kappa", "epl_deflection", "epl_kappa",
    "tnfw_G", "tnfw_deflection",
    "shear_deflection", "nfw_g", "nfw_deflection", "nfw_kappa", "point_mass_deflection",
    "total_deflection", "ray_shoot", "sersic_bn", "sersic", "surface_brightness",
    "gaussian", "core_sersic", "shapelets", "shapelet_phi", "shapelet_index", "component",
    "convolve_at", "convolve_same", "simulate_image", "simulate_unconvolved", "log_likelihood",
    "noise_variance", "chi2_gradient", "macro_vector", "macro_names", "basis_images", "linear_amplitudes",
    "splitmix64", "uniform", "pso", "pso_start", "pso_move", "pso_bests", "lbfgs",
    "PARITY_UNPINNED",
]
