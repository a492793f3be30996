"""Gradient of the chi^2 image log-likelihood (oracle, FP64).

The paper credits automatic differentiation with making gradient-based fitting
possible (L-BFGS through autodiff, "Improvements over lenstronomy in lens
modelling").  The oracle gradient is obtained the same way, but on the CPU in
FP64: the forward model of `simulate.py` is restated with torch float64 CPU
operations (same definitions and branch forms, checked equal to the NumPy
oracle by the pins), and torch.autograd differentiates

    log L = -1/2 sum_i (m_i - d_i)^2 w_i,   w_i = 1 / sigma_i^2 (data-based)

with respect to the lens, shear, Sersic and subhalo parameters.  It shares no
derivation with the GPU adjoint, which is written by hand.

Parameter vector per draw (`macro`):
  [theta_E, q, phi, cx, cy] of the SIE -- or, for an elliptical power-law
  main deflector, [theta_E, gamma, q, phi, cx, cy] of the EPL -- then
  [gamma1, gamma2] of the shear, then [amp, R_sersic, n_sersic, q, phi, cx, cy]
  for every source component, then the same seven for every lens-light
  component.
Subhalo gradients: (x, y, alpha_Rs) per subhalo, NFW or truncated NFW (Rs and
r_trunc are held fixed).  b_n is the Capaccioli fit 1.9992 n - 0.3271 (its
derivative in n is 1.9992).
"""
import math

import numpy as np

LN2 = math.log(2.0)


def _torch():
    import torch
    return torch


def main_kind(lens):
    """'epl' for an elliptical power-law main deflector, else 'sie'."""
    return "epl" if getattr(lens, "epl", None) is not None else "sie"


def main_size(kind):
    return 6 if kind == "epl" else 5


def macro_vector(lens, source, lens_light):
    if main_kind(lens) == "epl":
        e = lens.epl
        v = [e.theta_E, e.gamma, e.q, e.phi, e.cx, e.cy]
    else:
        v = [lens.sie.theta_E, lens.sie.q, lens.sie.phi, lens.sie.cx, lens.sie.cy]
    v += [lens.shear.gamma1, lens.shear.gamma2]
    for c in list(source) + list(lens_light):
        v += [c.amp, c.R_sersic, c.n_sersic, c.q, c.phi, c.cx, c.cy]
    return np.array(v, dtype=np.float64)


def macro_names(n_source, n_lens_light, kind="sie"):
    if kind == "epl":
        names = ["epl.theta_E", "epl.gamma", "epl.q", "epl.phi", "epl.cx", "epl.cy"]
    else:
        names = ["sie.theta_E", "sie.q", "sie.phi", "sie.cx", "sie.cy"]
    names += ["shear.gamma1", "shear.gamma2"]
    for tag, n in (("src", n_source), ("ll", n_lens_light)):
        for k in range(n):
            names += [f"{tag}{k}.{p}" for p in ("amp", "R_sersic", "n_sersic", "q", "phi", "cx", "cy")]
    return names


# ---------------------------------------------------------------- torch forward
def _sie(t, x, y, te, q, phi, cx, cy):
    c, s = t.cos(phi), t.sin(phi)
    dx, dy = x - cx, y - cy
    xp, yp = c * dx + s * dy, -s * dx + c * dy
    f = t.sqrt((1 - q) * (1 + q))
    psi2 = q * q * xp * xp + yp * yp
    pos = psi2 > 0                        # alpha = 0 at the centre (psi = 0)
    psi = t.sqrt(t.where(pos, psi2, t.ones_like(psi2)))
    pref = te * t.sqrt(q)
    if float(f.detach()) < 1e-3:
        zx, zy = f * xp / psi, f * yp / psi
        axp = pref * (xp / psi) * (1 - zx ** 2 / 3 + zx ** 4 / 5 - zx ** 6 / 7)
        ayp = pref * (yp / psi) * (1 + zy ** 2 / 3 + zy ** 4 / 5 + zy ** 6 / 7)
    else:
        axp = pref / f * t.atan(f * xp / psi)
        ayp = pref / f * t.atanh(f * yp / psi)
    axp = t.where(pos, axp, t.zeros_like(axp))
    ayp = t.where(pos, ayp, t.zeros_like(ayp))
    return c * axp - s * ayp, s * axp + c * ayp


def _epl(t, x, y, te, gamma, q, phi, cx, cy, terms=120):
    """EPL deflection (Tessore & Metcalf 2015), the closed form of the NumPy
    oracle with its Gauss hypergeometric factor 2F1(1, t/2; 2 - t/2; z),
    z = -(1-q)/(1+q) e^{2 i varphi}, summed as its power series
    sum_n z^n prod_{m<n} (t/2 + m)/(2 - t/2 + m) (|z| < 1; `terms` terms, so
    |z|^terms is below 1e-15 for q >= 0.3).  Complex numbers as (re, im)
    pairs; alpha = 0 at R = 0."""
    c, s = t.cos(phi), t.sin(phi)
    dx, dy = x - cx, y - cy
    xp, yp = c * dx + s * dy, -s * dx + c * dy
    tt = gamma - 1
    b = te * t.sqrt(q)
    R2 = q * q * xp * xp + yp * yp
    pos = R2 > 0
    R = t.sqrt(t.where(pos, R2, t.ones_like(R2)))
    er, ei = q * xp / R, yp / R                       # e^{i varphi}
    f = (1 - q) / (1 + q)
    zr, zi = -f * (er * er - ei * ei), -f * (2 * er * ei)
    sr, si = t.ones_like(R), t.zeros_like(R)           # partial sums of 2F1
    wr, wi = t.ones_like(R), t.zeros_like(R)           # current term
    for n in range(1, terms):
        k = (tt / 2 + n - 1) / (2 - tt / 2 + n - 1)
        wr, wi = k * (zr * wr - zi * wi), k * (zr * wi + zi * wr)
        sr, si = sr + wr, si + wi
    a = 2 * b / (1 + q) * (b / R) ** (tt - 1)
    axp = t.where(pos, a * (er * sr - ei * si), t.zeros_like(R))
    ayp = t.where(pos, a * (er * si + ei * sr), t.zeros_like(R))
    return c * axp - s * ayp, s * axp + c * ayp


def _nfw_F(t, X):
    """F(x) of the NFW with the oracle's branch forms (x > 0): the series in
    u = x^2 - 1 for |u| < 0.1, arccosh(1/x)/sqrt(1 - x^2) below, arccos(1/x)/
    sqrt(x^2 - 1) above; each branch on its own elements only."""
    u = X * X - 1
    near = u.abs() < 0.1
    lo = (X < 1) & ~near
    hi = (X > 1) & ~near
    out = t.zeros_like(X)
    if bool(near.any()):
        un = u[near]
        F = t.zeros_like(un)
        p = t.ones_like(un)
        for k in range(24):
            F = F + p / (2 * k + 1)
            p = p * (-un)
        out = out.index_put((near,), F)
    if bool(lo.any()):
        xl = X[lo]
        out = out.index_put((lo,), t.acosh(1 / xl) / t.sqrt(1 - xl * xl))
    if bool(hi.any()):
        xh = X[hi]
        out = out.index_put((hi,), t.acos(1 / xh) / t.sqrt(xh * xh - 1))
    return out


def _tnfw(t, x, y, rs, ars, rt, sx, sy):
    """Summed truncated-NFW deflection (Baltz, Marshall & Oguri 2009, the
    oracle's G(x, tau) with tau = r_trunc/Rs), alpha = alpha_Rs/(1 - ln 2)
    G/x (dx, dy)/r; x, y (P,), subhalo arrays (K,)."""
    dx = x[:, None] - sx[None, :]
    dy = y[:, None] - sy[None, :]
    r2 = dx * dx + dy * dy
    pos = r2 > 0
    r = t.sqrt(t.where(pos, r2, t.ones_like(r2)))
    X = r / rs[None, :]
    tau = (rt / rs)[None, :]
    t2 = tau * tau
    F = _nfw_F(t, X.reshape(-1)).reshape(X.shape)
    s = t.sqrt(t2 + X * X)
    L = t.log(X / (s + tau))
    G = t2 / (t2 + 1) ** 2 * ((t2 + 1 + 2 * (X * X - 1)) * F + math.pi * tau + (t2 - 1) * t.log(tau)
                              + s * (-math.pi + (t2 - 1) / tau * L))
    fac = t.where(pos, ars[None, :] / (1 - LN2) * G / X / r, t.zeros_like(r))
    return (fac * dx).sum(1), (fac * dy).sum(1)


def _nfw_g(t, X):
    """g(x) = ln(x/2) + F(x) with the oracle's branch forms (x > 0); each
    branch is evaluated on its own elements only."""
    u = X * X - 1
    near = u.abs() < 0.1
    small = (X < 0.5) & ~near
    lo = (X < 1) & ~near & ~small
    hi = (X > 1) & ~near
    out = t.zeros_like(X)
    if bool(near.any()):
        un = u[near]
        F = t.zeros_like(un)
        p = t.ones_like(un)
        for k in range(24):
            F = F + p / (2 * k + 1)
            p = p * (-un)
        out = out.index_put((near,), t.log(X[near] / 2) + F)
    if bool(small.any()):
        xs = X[small]
        x2 = xs * xs
        w = t.sqrt(1 - x2)
        L = t.log(xs / 2)
        out = out.index_put((small,), (-L * x2 / (1 + w) + t.log1p(-x2 / (2 * (1 + w)))) / w)
    if bool(lo.any()):
        xl = X[lo]
        out = out.index_put((lo,), t.log(xl / 2) + t.acosh(1 / xl) / t.sqrt(1 - xl * xl))
    if bool(hi.any()):
        xh = X[hi]
        out = out.index_put((hi,), t.log(xh / 2) + t.acos(1 / xh) / t.sqrt(xh * xh - 1))
    return out


def _nfw(t, x, y, rs, ars, sx, sy):
    """Summed NFW deflection; x, y (P,), subhalo arrays (K,)."""
    dx = x[:, None] - sx[None, :]
    dy = y[:, None] - sy[None, :]
    r2 = dx * dx + dy * dy
    pos = r2 > 0                          # alpha = 0 at r = 0
    r = t.sqrt(t.where(pos, r2, t.ones_like(r2)))
    X = r / rs[None, :]
    g = _nfw_g(t, X)
    fac = t.where(pos, ars[None, :] / (1 - LN2) * g / X / r, t.zeros_like(r))
    return (fac * dx).sum(1), (fac * dy).sum(1)


def _sersic(t, x, y, amp, R, n, q, phi, cx, cy):
    c, s = t.cos(phi), t.sin(phi)
    dx, dy = x - cx, y - cy
    xp, yp = c * dx + s * dy, -s * dx + c * dy
    Rr = t.sqrt(q * xp * xp + yp * yp / q)
    b = 1.9992 * n - 0.3271
    return amp * t.exp(-b * ((Rr / R) ** (1 / n) - 1))


def torch_forward(macro, sub_x, sub_y, sub_ars, sub_rs, grid, n_source, n_lens_light, psf, kind="sie",
                  sub_rt=None):
    """Model image (ny, nx) as a torch float64 tensor from torch parameters;
    kind 'epl' reads an EPL main deflector from the macro row, sub_rt (fixed
    truncation radii) makes the subhalos truncated NFWs."""
    t = _torch()
    g = grid
    d, s = float(g.pixel_scale), int(g.supersample)
    j = t.arange(g.nx, dtype=t.float64)
    i = t.arange(g.ny, dtype=t.float64)
    b = t.arange(s, dtype=t.float64)
    tx = (g.x0 + (j[None, :, None, None] - (g.nx - 1) / 2) * d
          + ((b[None, None, None, :] + 0.5) / s - 0.5) * d).expand(g.ny, g.nx, s, s).reshape(-1)
    ty = (g.y0 + (i[:, None, None, None] - (g.ny - 1) / 2) * d
          + ((b[None, None, :, None] + 0.5) / s - 0.5) * d).expand(g.ny, g.nx, s, s).reshape(-1)
    nm = main_size(kind)
    if kind == "epl":
        ax, ay = _epl(t, tx, ty, *[macro[k] for k in range(6)])
    else:
        ax, ay = _sie(t, tx, ty, *[macro[k] for k in range(5)])
    g1, g2 = macro[nm], macro[nm + 1]
    ax = ax + g1 * tx + g2 * ty
    ay = ay + g2 * tx - g1 * ty
    if sub_x is not None and sub_x.numel() > 0:
        if sub_rt is not None:
            nx_, ny_ = _tnfw(t, tx, ty, sub_rs, sub_ars, sub_rt, sub_x, sub_y)
        else:
            nx_, ny_ = _nfw(t, tx, ty, sub_rs, sub_ars, sub_x, sub_y)
        ax, ay = ax + nx_, ay + ny_
    bx, by = tx - ax, ty - ay
    sb = t.zeros_like(tx)
    o0 = nm + 2
    for k in range(n_source):
        sb = sb + _sersic(t, bx, by, *[macro[o0 + 7 * k + m] for m in range(7)])
    for k in range(n_lens_light):
        o = o0 + 7 * (n_source + k)
        sb = sb + _sersic(t, tx, ty, *[macro[o + m] for m in range(7)])
    img = d * d * sb.reshape(g.ny, g.nx, s * s).mean(-1)
    if psf is None:
        return img
    K = t.as_tensor(np.asarray(psf, dtype=np.float64))
    k = K.shape[0]
    # true convolution, zero padding, same size: conv2d correlates, so flip K
    w = t.flip(K, dims=(0, 1))[None, None]
    return t.nn.functional.conv2d(img[None, None], w, padding=(k - 1) // 2)[0, 0]


def chi2_gradient(scene, data, inv_var):
    """log L and its gradient for one scene.

    Returns (logL, g_macro (P,), g_sub (N, 3) for (x, y, alpha_Rs))."""
    t = _torch()
    lens = scene.lens
    macro = t.tensor(macro_vector(lens, scene.source, scene.lens_light), dtype=t.float64, requires_grad=True)
    nfw = lens.nfw
    srt = None
    if nfw is not None and nfw.n > 0:
        sx = t.tensor(np.asarray(nfw.x, np.float64), requires_grad=True)
        sy = t.tensor(np.asarray(nfw.y, np.float64), requires_grad=True)
        sa = t.tensor(np.asarray(nfw.alpha_Rs, np.float64), requires_grad=True)
        srs = t.tensor(np.asarray(nfw.Rs, np.float64))
        if getattr(nfw, "r_trunc", None) is not None:
            srt = t.tensor(np.asarray(nfw.r_trunc, np.float64))
    else:
        sx = sy = sa = srs = None
    m = torch_forward(macro, sx, sy, sa, srs, scene.grid, len(scene.source), len(scene.lens_light), scene.psf,
                      main_kind(lens), srt)
    dd = t.as_tensor(np.asarray(data, np.float64))
    w = t.as_tensor(np.asarray(inv_var, np.float64))
    logL = -0.5 * ((m - dd) ** 2 * w).sum()
    logL.backward()
    gm = macro.grad.numpy().copy()
    if sx is not None:
        gs = np.stack([sx.grad.numpy(), sy.grad.numpy(), sa.grad.numpy()], axis=1)
    else:
        gs = np.zeros((0, 3))
    return float(logL.detach()), gm, gs
