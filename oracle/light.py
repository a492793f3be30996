"""Elliptical Sersic surface brightness (oracle, FP64).

Step two of the paper's image simulation (image-simulation section) evaluates
the source light at the source-plane positions of the grid; the paper's flux
table lists SERSIC, SERSIC_ELLIPSE and SERSIC_ELLIPSE_Q_PHI.  The profile is Sersic
(1968):  I(R) = amp * exp(-b_n [(R/R_sersic)^(1/n) - 1]), with the amplitude
read as the surface brightness at R = R_sersic and the elliptical radius
R = sqrt(q x'^2 + y'^2/q) (product average; x' along the major axis at angle
phi about the component centre).
"""
import math

import numpy as np


def sersic_bn(n, exact=False):
    """b_n: Capaccioli (1989) linear fit 1.9992 n - 0.3271 by default; with
    `exact`, the root of P(2n, b) = 1/2 so that R_sersic is the half-light
    radius."""
    if exact:
        from scipy.special import gammaincinv
        return float(gammaincinv(2.0 * n, 0.5))
    return 1.9992 * n - 0.3271


def sersic(x, y, amp, R_sersic, n_sersic, q, phi, cx, cy, bn_exact=False):
    """Elliptical Sersic surface brightness at (x, y).  R = 0 gives amp e^b."""
    c, s = math.cos(phi), math.sin(phi)
    dx = np.asarray(x, dtype=np.float64) - cx
    dy = np.asarray(y, dtype=np.float64) - cy
    xp = c * dx + s * dy
    yp = -s * dx + c * dy
    R = np.sqrt(q * xp * xp + yp * yp / q)
    b = sersic_bn(n_sersic, bn_exact)
    return amp * np.exp(-b * ((R / R_sersic) ** (1.0 / n_sersic) - 1.0))


def surface_brightness(tx, ty, bx, by, source, lens_light, bn_exact=False):
    """Sub-pixel surface brightness: the source components evaluated at the
    traced positions beta plus the (unlensed) lens-light components evaluated at
    the image-plane positions theta."""
    out = np.zeros(np.shape(bx), dtype=np.float64)
    for c in source:
        out += sersic(bx, by, c.amp, c.R_sersic, c.n_sersic, c.q, c.phi, c.cx, c.cy, bn_exact)
    for c in lens_light:
        out += sersic(tx, ty, c.amp, c.R_sersic, c.n_sersic, c.q, c.phi, c.cx, c.cy, bn_exact)
    return out
