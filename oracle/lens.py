"""Deflection angles of the deflector profiles on the path (oracle, FP64).

Step one of the paper's image simulation (image-simulation section) maps every
image-plane angle to the source plane, which needs the deflection of each
deflector there; the paper's deflector table lists NIE/SIE, SIS, EPL, SHEAR,
NFW and TNFW among others.  It states no formula, so each profile here is the
standard closed form from the literature, named per function.  All angles are in
arcsec.  Single lens plane: beta = theta - sum_k alpha_k(theta).
"""
import math

import numpy as np

LN2 = math.log(2.0)


# --------------------------------------------------------------------------
# SIE / SIS  (Kormann, Schneider & Bartelmann 1994; Keeton 2001 catalogue)
# --------------------------------------------------------------------------
def _rotate_in(x, y, phi, cx, cy):
    c, s = math.cos(phi), math.sin(phi)
    dx = np.asarray(x, dtype=np.float64) - cx
    dy = np.asarray(y, dtype=np.float64) - cy
    return c * dx + s * dy, -s * dx + c * dy, c, s


def sie_kappa(x, y, theta_E, q, phi, cx, cy):
    """Convergence kappa = theta_E / (2 sqrt(q x'^2 + y'^2 / q)), the
    product-average normalisation in which theta_E is the Einstein radius of the
    equivalent circular model; x' lies along the major axis at angle phi."""
    xp, yp, _, _ = _rotate_in(x, y, phi, cx, cy)
    return theta_E / (2.0 * np.sqrt(q * xp * xp + yp * yp / q))


def sie_deflection(x, y, theta_E, q, phi, cx, cy):
    """SIE deflection for the convergence of `sie_kappa`.

    In the frame of the major axis, with f = sqrt(1 - q^2) and
    psi = sqrt(q^2 x'^2 + y'^2):
        alpha'_x = theta_E sqrt(q)/f * atan(f x'/psi)
        alpha'_y = theta_E sqrt(q)/f * atanh(f y'/psi)
    then rotated back by +phi.  For f < 1e-3 the atan/atanh ratios use their
    Taylor series (q = 1 gives the SIS, alpha = theta_E r_hat).  alpha = 0 at the
    centre (psi = 0).
    """
    xp, yp, c, s = _rotate_in(x, y, phi, cx, cy)
    f = math.sqrt((1.0 - q) * (1.0 + q))
    psi = np.sqrt(q * q * xp * xp + yp * yp)
    pref = theta_E * math.sqrt(q)
    safe = np.where(psi > 0.0, psi, 1.0)
    if f < 1e-3:
        zx = f * xp / safe
        zy = f * yp / safe
        axp = pref * (xp / safe) * (1.0 - zx ** 2 / 3.0 + zx ** 4 / 5.0 - zx ** 6 / 7.0)
        ayp = pref * (yp / safe) * (1.0 + zy ** 2 / 3.0 + zy ** 4 / 5.0 + zy ** 6 / 7.0)
    else:
        axp = pref / f * np.arctan(f * xp / safe)
        ayp = pref / f * np.arctanh(f * yp / safe)
    axp = np.where(psi > 0.0, axp, 0.0)
    ayp = np.where(psi > 0.0, ayp, 0.0)
    return c * axp - s * ayp, s * axp + c * ayp


# --------------------------------------------------------------------------
# EPL: elliptical power law  (Tessore & Metcalf 2015)
# --------------------------------------------------------------------------
def epl_kappa(x, y, theta_E, gamma, q, phi, cx, cy):
    """Convergence kappa = (3 - gamma)/2 * (theta_E / sqrt(q x'^2 + y'^2/q))^(gamma - 1):
    gamma is the slope of the 3-D density (gamma = 2 is the SIE of `sie_kappa`);
    theta_E is in the same product-average normalisation."""
    xp, yp, _, _ = _rotate_in(x, y, phi, cx, cy)
    return 0.5 * (3.0 - gamma) * (theta_E / np.sqrt(q * xp * xp + yp * yp / q)) ** (gamma - 1.0)


def epl_deflection(x, y, theta_E, gamma, q, phi, cx, cy):
    """EPL deflection for the convergence of `epl_kappa`, by the closed form of
    Tessore & Metcalf (2015) with the Gauss hypergeometric function.

    With t = gamma - 1, b = theta_E sqrt(q) and, in the frame of the major
    axis, the elliptical radius R = sqrt(q^2 x'^2 + y'^2) and angle
    e^{i varphi} = (q x' + i y') / R, the complex deflection is
        alpha' = 2 b / (1 + q) * (b / R)^(t - 1) * e^{i varphi}
                 * 2F1(1, t/2; 2 - t/2; -(1 - q)/(1 + q) e^{2 i varphi}),
    rotated back by +phi.  alpha = 0 at the centre (R = 0) and for theta_E = 0.
    """
    from scipy.special import hyp2f1
    xp, yp, c, s = _rotate_in(x, y, phi, cx, cy)
    t = gamma - 1.0
    b = theta_E * math.sqrt(q)
    R = np.sqrt(q * q * xp * xp + yp * yp)
    ok = (R > 0.0) & (theta_E > 0.0)
    safe = np.where(ok, R, 1.0)
    eiv = (q * xp + 1j * yp) / safe
    z = -(1.0 - q) / (1.0 + q) * eiv * eiv
    with np.errstate(invalid="ignore", divide="ignore"):
        a = 2.0 * b / (1.0 + q) * (b / safe) ** (t - 1.0) * eiv * hyp2f1(1.0, 0.5 * t, 2.0 - 0.5 * t, z)
    axp = np.where(ok, a.real, 0.0)
    ayp = np.where(ok, a.imag, 0.0)
    return c * axp - s * ayp, s * axp + c * ayp


# --------------------------------------------------------------------------
# external shear
# --------------------------------------------------------------------------
def shear_deflection(x, y, gamma1, gamma2):
    """External shear about the origin, from the potential
    psi = gamma1 (x^2 - y^2)/2 + gamma2 x y:  alpha = (g1 x + g2 y, g2 x - g1 y)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return gamma1 * x + gamma2 * y, gamma2 * x - gamma1 * y


# --------------------------------------------------------------------------
# NFW  (Bartelmann 1996; Wright & Brainerd 2000; Golse & Kneib 2002)
# --------------------------------------------------------------------------
def _F_series(u, terms=24):
    """F as a power series in u = x^2 - 1: sum_k (-u)^k / (2k+1), valid on
    both sides of x = 1 (it is atan(sqrt(u))/sqrt(u) for u > 0 and
    atanh(sqrt(-u))/sqrt(-u) for u < 0)."""
    acc = np.zeros_like(u)
    p = np.ones_like(u)
    for k in range(terms):
        acc = acc + p / (2 * k + 1)
        p = p * (-u)
    return acc


def _nfw_F(X):
    """F(x) = arccosh(1/x)/sqrt(1-x^2) (x<1), 1 (x=1), arccos(1/x)/sqrt(x^2-1) (x>1)."""
    X = np.asarray(X, dtype=np.float64)
    u = X * X - 1.0
    out = np.empty_like(X)
    near = np.abs(u) < 0.1
    lo = (X < 1.0) & ~near
    hi = (X > 1.0) & ~near
    out[near] = _F_series(u[near])
    xl = X[lo]
    out[lo] = np.arccosh(1.0 / xl) / np.sqrt(1.0 - xl * xl)
    xh = X[hi]
    out[hi] = np.arccos(1.0 / xh) / np.sqrt(xh * xh - 1.0)
    return out


def nfw_g(X):
    """g(x) = ln(x/2) + F(x), the dimensionless enclosed projected NFW mass
    (x = r/Rs), evaluated without cancellation:
      x < 0.5:       g = [-L x^2/(1+w) + log1p(-x^2/(2(1+w)))]/w,
                     L = ln(x/2), w = sqrt(1-x^2)
      |x^2-1| < 0.1: F by its power series in x^2-1
      otherwise:     the direct form.
    g(0) = 0."""
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros_like(X)
    small = (X < 0.5) & (X > 0.0)
    rest = X >= 0.5
    xs = X[small]
    x2 = xs * xs
    w = np.sqrt(1.0 - x2)
    L = np.log(xs / 2.0)
    out[small] = (-L * x2 / (1.0 + w) + np.log1p(-x2 / (2.0 * (1.0 + w)))) / w
    xr = X[rest]
    out[rest] = np.log(xr / 2.0) + _nfw_F(xr)
    return out


def nfw_kappa(x, y, Rs, alpha_Rs, cx, cy):
    """NFW convergence kappa = 2 kappa_s (1 - F(x)) / (x^2 - 1), with
    kappa_s = alpha_Rs / (4 Rs (1 - ln 2)); kappa(x=1) = 2 kappa_s / 3."""
    r = np.hypot(np.asarray(x, dtype=np.float64) - cx, np.asarray(y, dtype=np.float64) - cy)
    X = r / Rs
    ks = alpha_Rs / (4.0 * Rs * (1.0 - LN2))
    u = X * X - 1.0
    out = np.empty_like(X)
    near = np.abs(u) < 0.1
    un = u[near]
    # (1 - F)/u = sum_{k>=1} (-1)^(k+1) u^(k-1) / (2k+1)
    acc = np.zeros_like(un)
    p = np.ones_like(un)
    for k in range(1, 26):
        acc = acc + (1.0 if k % 2 == 1 else -1.0) * p / (2 * k + 1)
        p = p * un
    out[near] = 2.0 * ks * acc
    Xf = X[~near]
    out[~near] = 2.0 * ks * (1.0 - _nfw_F(Xf)) / (Xf * Xf - 1.0)
    return out


def nfw_deflection(x, y, Rs, alpha_Rs, cx, cy, chunk_points=4096, chunk_sub=1024):
    """Sum of NFW deflections over subhalos k:
        alpha_k = alpha_Rs,k / (1 - ln 2) * g(r/Rs,k) / (r/Rs,k) * (dx, dy)/r,
    so that |alpha_k(r = Rs,k)| = alpha_Rs,k; alpha_k = 0 at r = 0.
    `Rs, alpha_Rs, cx, cy` are 1-D arrays (or scalars); x, y any shape."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    shape = x.shape
    xf = x.reshape(-1)
    yf = y.reshape(-1)
    Rs = np.atleast_1d(np.asarray(Rs, dtype=np.float64))
    aRs = np.atleast_1d(np.asarray(alpha_Rs, dtype=np.float64))
    cx = np.atleast_1d(np.asarray(cx, dtype=np.float64))
    cy = np.atleast_1d(np.asarray(cy, dtype=np.float64))
    ax = np.zeros_like(xf)
    ay = np.zeros_like(yf)
    nsub = Rs.shape[0]
    for p0 in range(0, xf.shape[0], chunk_points):
        px = xf[p0:p0 + chunk_points, None]
        py = yf[p0:p0 + chunk_points, None]
        sx = np.zeros(px.shape[0])
        sy = np.zeros(px.shape[0])
        for k0 in range(0, nsub, chunk_sub):
            sl = slice(k0, k0 + chunk_sub)
            dx = px - cx[None, sl]
            dy = py - cy[None, sl]
            r = np.hypot(dx, dy)
            X = r / Rs[None, sl]
            g = nfw_g(X)
            with np.errstate(invalid="ignore", divide="ignore"):
                fac = np.where(r > 0.0, aRs[None, sl] / (1.0 - LN2) * g / X / r, 0.0)
            sx += np.sum(fac * dx, axis=1)
            sy += np.sum(fac * dy, axis=1)
        ax[p0:p0 + chunk_points] = sx
        ay[p0:p0 + chunk_points] = sy
    return ax.reshape(shape), ay.reshape(shape)


# --------------------------------------------------------------------------
# TNFW: truncated NFW  (Baltz, Marshall & Oguri 2009, truncation exponent 1)
# --------------------------------------------------------------------------
def tnfw_G(X, tau):
    """Projected mass inside x = R/Rs of the density
    rho_NFW(r) tau^2 / (tau^2 + (r/Rs)^2), tau = r_trunc/Rs, in the units in
    which the untruncated profile's is `nfw_g`:
        G = tau^2/(tau^2+1)^2 [ (tau^2 + 1 + 2(x^2 - 1)) F(x) + pi tau
                                + (tau^2 - 1) ln tau
                                + sqrt(tau^2 + x^2) (-pi + (tau^2 - 1)/tau L(x)) ],
        L(x) = ln( x / (sqrt(tau^2 + x^2) + tau) ),
    with F of `nfw_g`.  X and tau broadcast."""
    X = np.asarray(X, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    X, tau = np.broadcast_arrays(X, tau)
    t2 = tau * tau
    s = np.sqrt(t2 + X * X)
    F = _nfw_F(X.reshape(-1)).reshape(X.shape)
    with np.errstate(divide="ignore", invalid="ignore"):
        L = np.log(X / (s + tau))
        return t2 / (t2 + 1.0) ** 2 * ((t2 + 1.0 + 2.0 * (X * X - 1.0)) * F + np.pi * tau
                                       + (t2 - 1.0) * np.log(tau) + s * (-np.pi + (t2 - 1.0) / tau * L))


def tnfw_deflection(x, y, Rs, alpha_Rs, r_trunc, cx, cy, chunk_points=4096, chunk_sub=1024):
    """Sum of TNFW deflections over subhalos k, normalised like the NFW (alpha_Rs
    is the untruncated profile's deflection at r = Rs, so both share rho_0):
        alpha_k = alpha_Rs,k / (1 - ln 2) * G(r/Rs,k, tau_k) / (r/Rs,k) * (dx, dy)/r,
    tau_k = r_trunc,k / Rs,k; alpha_k = 0 at r = 0."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    shape = x.shape
    xf = x.reshape(-1)
    yf = y.reshape(-1)
    Rs = np.atleast_1d(np.asarray(Rs, dtype=np.float64))
    aRs = np.atleast_1d(np.asarray(alpha_Rs, dtype=np.float64))
    tau = np.atleast_1d(np.asarray(r_trunc, dtype=np.float64)) / Rs
    cx = np.atleast_1d(np.asarray(cx, dtype=np.float64))
    cy = np.atleast_1d(np.asarray(cy, dtype=np.float64))
    ax = np.zeros_like(xf)
    ay = np.zeros_like(yf)
    nsub = Rs.shape[0]
    for p0 in range(0, xf.shape[0], chunk_points):
        px = xf[p0:p0 + chunk_points, None]
        py = yf[p0:p0 + chunk_points, None]
        sx = np.zeros(px.shape[0])
        sy = np.zeros(px.shape[0])
        for k0 in range(0, nsub, chunk_sub):
            sl = slice(k0, k0 + chunk_sub)
            dx = px - cx[None, sl]
            dy = py - cy[None, sl]
            r = np.hypot(dx, dy)
            X = r / Rs[None, sl]
            G = tnfw_G(np.where(r > 0.0, X, 1.0), tau[None, sl])
            with np.errstate(invalid="ignore", divide="ignore"):
                fac = np.where(r > 0.0, aRs[None, sl] / (1.0 - LN2) * G / X / r, 0.0)
            sx += np.sum(fac * dx, axis=1)
            sy += np.sum(fac * dy, axis=1)
        ax[p0:p0 + chunk_points] = sx
        ay[p0:p0 + chunk_points] = sy
    return ax.reshape(shape), ay.reshape(shape)


# --------------------------------------------------------------------------
# point mass (test profile)
# --------------------------------------------------------------------------
def point_mass_deflection(x, y, theta_E, cx, cy):
    """Sum of point-mass deflections alpha = theta_E^2 (dx, dy)/r^2 (0 at r = 0)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    ax = np.zeros_like(x)
    ay = np.zeros_like(y)
    for te, px, py in zip(np.atleast_1d(theta_E), np.atleast_1d(cx), np.atleast_1d(cy)):
        dx = x - float(px)
        dy = y - float(py)
        r2 = dx * dx + dy * dy
        with np.errstate(invalid="ignore", divide="ignore"):
            fac = np.where(r2 > 0.0, float(te) ** 2 / r2, 0.0)
        ax += fac * dx
        ay += fac * dy
    return ax, ay


# --------------------------------------------------------------------------
# ray shooting
# --------------------------------------------------------------------------
def total_deflection(x, y, lens):
    """Sum of the deflections of every deflector in `lens` (attributes sie,
    epl, shear, nfw, point_masses; any may be None or absent)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    ax = np.zeros_like(x)
    ay = np.zeros_like(y)
    if getattr(lens, "sie", None) is not None:
        s = lens.sie
        dx, dy = sie_deflection(x, y, s.theta_E, s.q, s.phi, s.cx, s.cy)
        ax += dx
        ay += dy
    if getattr(lens, "epl", None) is not None:
        e = lens.epl
        dx, dy = epl_deflection(x, y, e.theta_E, e.gamma, e.q, e.phi, e.cx, e.cy)
        ax += dx
        ay += dy
    if getattr(lens, "shear", None) is not None:
        dx, dy = shear_deflection(x, y, lens.shear.gamma1, lens.shear.gamma2)
        ax += dx
        ay += dy
    nfw = getattr(lens, "nfw", None)
    if nfw is not None and nfw.x.shape[0] > 0 and getattr(nfw, "r_trunc", None) is not None:
        dx, dy = tnfw_deflection(x, y, nfw.Rs, nfw.alpha_Rs, nfw.r_trunc, nfw.x, nfw.y)
        ax += dx
        ay += dy
    elif nfw is not None and nfw.x.shape[0] > 0:
        dx, dy = nfw_deflection(x, y, nfw.Rs, nfw.alpha_Rs, nfw.x, nfw.y)
        ax += dx
        ay += dy
    pm = getattr(lens, "point_masses", None)
    if pm is not None and np.size(pm.x) > 0:
        dx, dy = point_mass_deflection(x, y, pm.theta_E, pm.x, pm.y)
        ax += dx
        ay += dy
    return ax, ay


def ray_shoot(x, y, lens):
    """Source-plane position beta = theta - alpha(theta) (single lens plane)."""
    ax, ay = total_deflection(x, y, lens)
    return np.asarray(x, dtype=np.float64) - ax, np.asarray(y, dtype=np.float64) - ay
