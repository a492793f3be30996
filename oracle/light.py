"""Surface brightness of the light profiles (oracle, FP64).

Step two of the paper's image simulation (image-simulation section) evaluates
the source light at the source-plane positions of the grid; the paper's flux
table lists SERSIC (and its elliptical forms), CORE_SERSIC, GAUSSIAN(_ELLIPSE),
MULTI_GAUSSIAN(_ELLIPSE) and SHAPELETS.  It states no formula; the readings:

* Sersic (1968): I(R) = amp * exp(-b_n [(R/R_sersic)^(1/n) - 1]), the
  amplitude read as the surface brightness at R = R_sersic, with the
  elliptical radius R = sqrt(q x'^2 + y'^2/q) (product average; x' along the
  major axis at angle phi about the component centre).
* Gaussian: I = amp / (2 pi sigma^2) exp(-R^2 / (2 sigma^2)) with the same R,
  so amp is the total flux (the map (sqrt(q) x', y'/sqrt(q)) keeps areas).
  A multi-Gaussian is a list of them.
* Core-Sersic (Graham et al. 2003; Trujillo et al. 2004):
  I = amp (1 + (R_b/R)^alpha)^(gamma/alpha)
          exp(-b_n [((R^alpha + R_b^alpha)/R_sersic^alpha)^(1/(n alpha)) - 1]),
  normalised so that R_b -> 0 gives the Sersic above; R is floored at
  1e-6 R_b where the inner power law diverges.
* Shapelets (Refregier 2003): I = sum over n1 + n2 <= n_max of
  c_{n1 n2} B_{n1}(x) B_{n2}(y), B_n(x) = beta^(-1/2) phi_n((x - cx)/beta),
  phi_n(u) = (2^n sqrt(pi) n!)^(-1/2) H_n(u) exp(-u^2/2) (Hermite H_n), an
  orthonormal basis of the plane; coefficients ordered by n = n1 + n2, then
  n2 = 0..n (n1 = n - n2).
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


def _elliptical_R2(x, y, q, phi, cx, cy):
    c, s = math.cos(phi), math.sin(phi)
    dx = np.asarray(x, dtype=np.float64) - cx
    dy = np.asarray(y, dtype=np.float64) - cy
    xp = c * dx + s * dy
    yp = -s * dx + c * dy
    return q * xp * xp + yp * yp / q


def gaussian(x, y, amp, sigma, q, phi, cx, cy):
    """Elliptical Gaussian of total flux amp."""
    R2 = _elliptical_R2(x, y, q, phi, cx, cy)
    return amp / (2.0 * math.pi * sigma * sigma) * np.exp(-R2 / (2.0 * sigma * sigma))


def core_sersic(x, y, amp, R_sersic, R_b, n_sersic, gamma, alpha, q, phi, cx, cy, bn_exact=False):
    """Elliptical core-Sersic profile (see the module docstring)."""
    R = np.sqrt(_elliptical_R2(x, y, q, phi, cx, cy))
    R = np.maximum(R, 1e-6 * R_b)
    b = sersic_bn(n_sersic, bn_exact)
    inner = (1.0 + (R_b / R) ** alpha) ** (gamma / alpha)
    outer = ((R ** alpha + R_b ** alpha) / R_sersic ** alpha) ** (1.0 / (n_sersic * alpha))
    return amp * inner * np.exp(-b * (outer - 1.0))


def shapelet_phi(n, u):
    """phi_n(u) = (2^n sqrt(pi) n!)^(-1/2) H_n(u) exp(-u^2/2) from SciPy's
    Hermite polynomial."""
    from scipy.special import eval_hermite
    u = np.asarray(u, dtype=np.float64)
    return eval_hermite(n, u) * np.exp(-0.5 * u * u) / math.sqrt(2.0 ** n * math.sqrt(math.pi) * math.factorial(n))


def shapelet_index(n1, n2):
    n = n1 + n2
    return n * (n + 1) // 2 + n2


def shapelets(x, y, coeff, n_max, beta, cx, cy):
    u = (np.asarray(x, dtype=np.float64) - cx) / beta
    v = (np.asarray(y, dtype=np.float64) - cy) / beta
    out = np.zeros(np.broadcast(u, v).shape)
    for n1 in range(n_max + 1):
        pu = shapelet_phi(n1, u)
        for n2 in range(n_max + 1 - n1):
            out += coeff[shapelet_index(n1, n2)] * pu * shapelet_phi(n2, v) / beta
    return out


def component(x, y, c, bn_exact=False):
    """One light component of any profile (dispatch on its fields)."""
    if hasattr(c, "coeff"):
        return shapelets(x, y, np.asarray(c.coeff, dtype=np.float64), c.n_max, c.beta, c.cx, c.cy)
    if hasattr(c, "sigma"):
        return gaussian(x, y, c.amp, c.sigma, c.q, c.phi, c.cx, c.cy)
    if hasattr(c, "R_b"):
        return core_sersic(x, y, c.amp, c.R_sersic, c.R_b, c.n_sersic, c.gamma, c.alpha, c.q, c.phi, c.cx, c.cy,
                           bn_exact)
    return sersic(x, y, c.amp, c.R_sersic, c.n_sersic, c.q, c.phi, c.cx, c.cy, bn_exact)


def surface_brightness(tx, ty, bx, by, source, lens_light, bn_exact=False):
    """Sub-pixel surface brightness: the source components evaluated at the
    traced positions beta plus the (unlensed) lens-light components evaluated at
    the image-plane positions theta."""
    out = np.zeros(np.shape(bx), dtype=np.float64)
    for c in source:
        out += component(bx, by, c, bn_exact)
    for c in lens_light:
        out += component(tx, ty, c, bn_exact)
    return out
