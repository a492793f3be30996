"""Seeded synthetic inputs for the lensed-image simulation.

This module only *draws* inputs: grids, macro-lens parameters, subhalo tables,
light components and pixelised PSFs, with the shapes and distributions of the
paper's workloads (a three-step simulation: ray-tracing, source surface
brightness, PSF convolution; "Improvements over lenstronomy in image
simulation").  It computes none of the method's arithmetic: no deflection, no
surface brightness, no convolution.  Both the FP64 oracle and the HIP path
consume exactly the arrays produced here.

Every floating-point parameter is rounded to FP32 before it is handed out, so the
oracle (which promotes to FP64) and the FP32 kernels see identical inputs and
input quantisation is never counted as kernel error.

Readings (the paper fixes none of these; they only shape the synthetic inputs):

* Subhalo masses map to the NFW (Rs, alpha_Rs) parameterisation through a flat
  LCDM cosmology (H0 = 70 km/s/Mpc, Om = 0.3), lens redshift 0.5, source
  redshift 1.5, M200 halos with concentration c200 = 15 (M / 1e8 Msun)^-0.1.
* Positions "uniform within R" are uniform in the disk of radius R about the
  main-lens centre.
* A "log-uniform subhalo count in [0, N]" is floor(10^U(0, log10(N + 1))) - 1.
* PSFs are point-sampled at pixel centres and normalised to unit sum.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Grid", "SIE", "Shear", "NFWTable", "PointMasses", "Sersic", "Lens", "Scene",
    "f32", "gaussian_psf", "airy_mix_psf", "nfw_params_from_mass",
    "config1_scene", "config2_scene", "config4_scene", "config5_scene",
    "config3_requests", "random_points", "noisy_image", "config4_draws",
]


def f32(v: float) -> float:
    """Round a Python float to the nearest FP32 value (returned as float)."""
    return float(np.float32(v))


# --------------------------------------------------------------------------
# plain containers (no arithmetic)
# --------------------------------------------------------------------------
@dataclass
class Grid:
    """Image grid: nx columns along +x, ny rows along +y, square pixels of
    `pixel_scale` arcsec centred on (x0, y0); `supersample` sub-pixels per axis."""
    nx: int
    ny: int
    pixel_scale: float
    x0: float = 0.0
    y0: float = 0.0
    supersample: int = 1


@dataclass
class SIE:
    """Singular isothermal ellipsoid: Einstein radius theta_E (arcsec), axis
    ratio q in (0, 1], position angle phi (rad, CCW from +x to the major axis),
    centre (cx, cy)."""
    theta_E: float
    q: float
    phi: float
    cx: float
    cy: float


@dataclass
class EPL:
    """Elliptical power-law main deflector: Einstein radius theta_E (arcsec),
    3-D density slope gamma in (1, 3) (2 = SIE), axis ratio q, position angle
    phi, centre (cx, cy)."""
    theta_E: float
    gamma: float
    q: float
    phi: float
    cx: float
    cy: float


@dataclass
class Shear:
    """External shear (gamma1, gamma2), centred on the coordinate origin."""
    gamma1: float
    gamma2: float


@dataclass
class NFWTable:
    """NFW subhalos as a structure of FP32 arrays (arcsec): centres (x, y),
    scale radius Rs and alpha_Rs, the deflection at r = Rs; with `r_trunc`
    (truncation radii) they are truncated NFW (TNFW) subhalos of the same
    inner density."""
    x: np.ndarray
    y: np.ndarray
    Rs: np.ndarray
    alpha_Rs: np.ndarray
    r_trunc: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class PointMasses:
    """Point lenses (a test-only profile): centres (x, y), Einstein radius."""
    x: np.ndarray
    y: np.ndarray
    theta_E: np.ndarray


@dataclass
class Sersic:
    """Elliptical Sersic light component: amplitude = surface brightness at
    R = R_sersic, index n_sersic, axis ratio q, angle phi, centre (cx, cy)."""
    amp: float
    R_sersic: float
    n_sersic: float
    q: float
    phi: float
    cx: float
    cy: float


@dataclass
class Gaussian:
    """Elliptical Gaussian light of total flux amp, width sigma (arcsec)."""
    amp: float
    sigma: float
    q: float
    phi: float
    cx: float
    cy: float


@dataclass
class CoreSersic:
    """Core-Sersic light: Sersic outside the break radius R_b, inner power
    law of slope gamma, transition sharpness alpha."""
    amp: float
    R_sersic: float
    R_b: float
    n_sersic: float
    gamma: float
    alpha: float
    q: float
    phi: float
    cx: float
    cy: float


@dataclass
class Shapelets:
    """Cartesian shapelets up to order n_max, scale beta, centre (cx, cy);
    (n_max + 1)(n_max + 2)/2 coefficients ordered by n = n1 + n2, then n2."""
    n_max: int
    beta: float
    cx: float
    cy: float
    coeff: np.ndarray


@dataclass
class Lens:
    sie: Optional[SIE] = None
    epl: Optional[EPL] = None
    shear: Optional[Shear] = None
    nfw: Optional[NFWTable] = None
    point_masses: Optional[PointMasses] = None


@dataclass
class Scene:
    """Everything one simulated image needs."""
    grid: Grid
    lens: Lens
    source: List[Sersic] = field(default_factory=list)
    lens_light: List[Sersic] = field(default_factory=list)
    psf: Optional[np.ndarray] = None          # (k, k) float32, odd k, unit sum
    bn_exact: bool = False


# --------------------------------------------------------------------------
# PSFs
# --------------------------------------------------------------------------
def _psf_radius(k: int) -> np.ndarray:
    c = (k - 1) / 2.0
    a = np.arange(k, dtype=np.float64) - c
    return np.hypot(a[None, :], a[:, None])


def gaussian_psf(k: int, fwhm_px: float, truncate_sigma: Optional[float] = None) -> np.ndarray:
    """Odd k x k Gaussian kernel point-sampled at pixel centres, optionally set
    to zero beyond `truncate_sigma` sigma, normalised to unit sum (FP32)."""
    if k % 2 != 1:
        raise ValueError("PSF size must be odd")
    sigma = fwhm_px / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    r = _psf_radius(k)
    ker = np.exp(-0.5 * (r / sigma) ** 2)
    if truncate_sigma is not None:
        ker[r > truncate_sigma * sigma] = 0.0
    ker /= ker.sum()
    ker = ker.astype(np.float32)
    return (ker / ker.sum(dtype=np.float64)).astype(np.float32)


def airy_mix_psf(k: int, fwhm_px: float, first_zero_px: float, noise: float,
                 rng: np.random.Generator) -> np.ndarray:
    """0.9 Gaussian(FWHM) + 0.1 Airy pattern [2 J1(z)/z]^2 with its first zero
    at `first_zero_px`, multiplied by (1 + noise N(0,1)), clipped at zero and
    normalised (FP32)."""
    from scipy.special import j1
    if k % 2 != 1:
        raise ValueError("PSF size must be odd")
    r = _psf_radius(k)
    sigma = fwhm_px / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    g = np.exp(-0.5 * (r / sigma) ** 2)
    g /= g.sum()
    z = 3.8317059702075125 * r / first_zero_px
    with np.errstate(invalid="ignore", divide="ignore"):
        airy = np.where(z > 0, (2.0 * j1(z) / np.where(z > 0, z, 1.0)) ** 2, 1.0)
    airy /= airy.sum()
    ker = 0.9 * g + 0.1 * airy
    ker *= 1.0 + noise * rng.standard_normal(ker.shape)
    ker = np.clip(ker, 0.0, None)
    ker = (ker / ker.sum()).astype(np.float32)
    return (ker / ker.sum(dtype=np.float64)).astype(np.float32)


# --------------------------------------------------------------------------
# subhalo masses -> NFW (Rs, alpha_Rs)
# --------------------------------------------------------------------------
_C_KM_S = 299792.458
_G_MPC_MSUN = 4.30091727e-9           # G in Mpc (km/s)^2 / Msun
_ARCSEC = math.pi / (180.0 * 3600.0)


def _comoving(z1: float, z2: float, om: float) -> float:
    from scipy.integrate import quad
    val, _ = quad(lambda z: 1.0 / math.sqrt(om * (1 + z) ** 3 + (1 - om)), z1, z2)
    return val


def nfw_params_from_mass(m200: np.ndarray, z_lens: float = 0.5, z_source: float = 1.5,
                         h0: float = 70.0, om: float = 0.3):
    """(Rs, alpha_Rs) in arcsec for M200 halos (Msun) with
    c200 = 15 (M/1e8)^-0.1 in flat LCDM.  Generator only: the simulation takes
    (Rs, alpha_Rs) as given."""
    m = np.asarray(m200, dtype=np.float64)
    dh = _C_KM_S / h0                                   # Hubble distance, Mpc
    d_l = dh * _comoving(0.0, z_lens, om) / (1 + z_lens)
    d_s = dh * _comoving(0.0, z_source, om) / (1 + z_source)
    d_ls = dh * _comoving(z_lens, z_source, om) / (1 + z_source)
    hz = h0 * math.sqrt(om * (1 + z_lens) ** 3 + (1 - om))  # km/s/Mpc
    rho_crit = 3.0 * hz * hz / (8.0 * math.pi * _G_MPC_MSUN)  # Msun / Mpc^3
    c = 15.0 * (m / 1e8) ** -0.1
    r200 = (3.0 * m / (4.0 * math.pi * 200.0 * rho_crit)) ** (1.0 / 3.0)
    rs = r200 / c                                        # Mpc
    rho_s = (200.0 / 3.0) * rho_crit * c ** 3 / (np.log1p(c) - c / (1.0 + c))
    sigma_crit = _C_KM_S ** 2 / (4.0 * math.pi * _G_MPC_MSUN) * d_s / (d_l * d_ls)
    kappa_s = rho_s * rs / sigma_crit
    rs_arcsec = rs / d_l / _ARCSEC
    alpha_rs = 4.0 * kappa_s * rs_arcsec * (1.0 - math.log(2.0))
    return rs_arcsec, alpha_rs


# --------------------------------------------------------------------------
# parameter priors
# --------------------------------------------------------------------------
def _rngs(seed: int, n: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


def _macro(rng: np.random.Generator):
    sie = SIE(theta_E=f32(rng.uniform(0.8, 1.5)), q=f32(rng.uniform(0.6, 1.0)),
              phi=f32(rng.uniform(0.0, math.pi)), cx=f32(rng.normal(0.0, 0.05)),
              cy=f32(rng.normal(0.0, 0.05)))
    shear = Shear(gamma1=f32(rng.normal(0.0, 0.03)), gamma2=f32(rng.normal(0.0, 0.03)))
    return sie, shear


def _macro_epl(rng: np.random.Generator):
    epl = EPL(theta_E=f32(rng.uniform(0.8, 1.5)), gamma=f32(rng.uniform(1.8, 2.2)),
              q=f32(rng.uniform(0.6, 1.0)), phi=f32(rng.uniform(0.0, math.pi)),
              cx=f32(rng.normal(0.0, 0.05)), cy=f32(rng.normal(0.0, 0.05)))
    shear = Shear(gamma1=f32(rng.normal(0.0, 0.03)), gamma2=f32(rng.normal(0.0, 0.03)))
    return epl, shear


def _source(rng: np.random.Generator, amp: float) -> Sersic:
    return Sersic(amp=f32(amp), R_sersic=f32(rng.uniform(0.1, 0.4)),
                  n_sersic=f32(rng.uniform(1.0, 4.0)), q=f32(rng.uniform(0.6, 1.0)),
                  phi=f32(rng.uniform(0.0, math.pi)), cx=f32(rng.normal(0.0, 0.1)),
                  cy=f32(rng.normal(0.0, 0.1)))


def _lens_light(rng: np.random.Generator, sie) -> Sersic:
    return Sersic(amp=f32(5.0), R_sersic=f32(rng.uniform(0.5, 1.5)),
                  n_sersic=f32(rng.uniform(2.0, 4.0)), q=f32(rng.uniform(0.6, 1.0)),
                  phi=f32(rng.uniform(0.0, math.pi)), cx=sie.cx, cy=sie.cy)


def _subhalos(rng: np.random.Generator, n: int, m_lo: float, m_hi: float,
              radius: float, cx: float, cy: float) -> NFWTable:
    logm = rng.uniform(math.log10(m_lo), math.log10(m_hi), size=n)
    rs, ars = nfw_params_from_mass(10.0 ** logm)
    rad = radius * np.sqrt(rng.uniform(0.0, 1.0, size=n))
    ang = rng.uniform(0.0, 2.0 * math.pi, size=n)
    x = cx + rad * np.cos(ang)
    y = cy + rad * np.sin(ang)
    return NFWTable(x=x.astype(np.float32), y=y.astype(np.float32),
                    Rs=rs.astype(np.float32), alpha_Rs=ars.astype(np.float32))


# --------------------------------------------------------------------------
# workload configurations
# --------------------------------------------------------------------------
def config1_scene(draw: int = 0, seed: int = 1001) -> Scene:
    """Plain-method case: 64x64 px at 0.05"/px, no supersampling; SIE + shear;
    one Sersic source of amplitude 10; 11x11 Gaussian PSF (FWHM 0.1",
    truncated at 5 sigma).  `draw` selects one of the seeded draws."""
    r_macro, r_src = _rngs(seed * 1000 + draw, 2)
    sie, shear = _macro(r_macro)
    src = _source(r_src, 10.0)
    grid = Grid(nx=64, ny=64, pixel_scale=0.05, supersample=1)
    psf = gaussian_psf(11, 0.1 / 0.05, truncate_sigma=5.0)
    return Scene(grid=grid, lens=Lens(sie=sie, shear=shear), source=[src], psf=psf)


def config2_scene(seed: int = 1002, n_sub: int = 10000, npix: int = 200,
                  supersample: int = 3, psf_size: int = 41) -> Scene:
    """Single-image headline case: 200x200 px at 0.05"/px, supersampling 3;
    SIE + shear + 10,000 NFW subhalos (M log-uniform in [1e6, 1e9] Msun,
    uniform within 3" of the lens centre); one lens-light and two source Sersic
    components; 41x41 Gaussian + Airy-ring PSF with 1% seeded noise."""
    r_macro, r_sub, r_ll, r_s1, r_s2, r_psf = _rngs(seed, 6)
    sie, shear = _macro(r_macro)
    nfw = _subhalos(r_sub, n_sub, 1e6, 1e9, 3.0, sie.cx, sie.cy)
    ll = _lens_light(r_ll, sie)
    srcs = [_source(r_s1, 10.0), _source(r_s2, 5.0)]
    grid = Grid(nx=npix, ny=npix, pixel_scale=0.05, supersample=supersample)
    psf = airy_mix_psf(psf_size, 2.0, 3.0, 0.01, r_psf)
    return Scene(grid=grid, lens=Lens(sie=sie, shear=shear, nfw=nfw), source=srcs,
                 lens_light=[ll], psf=psf)


def epl_scene(seed: int = 1006, n_sub: int = 10000, npix: int = 200,
              supersample: int = 3, psf_size: int = 41) -> Scene:
    """The headline image with an elliptical power-law main deflector in place
    of the SIE (slope gamma uniform in [1.8, 2.2], the other priors as the
    SIE's): 200x200 px at 0.05"/px, s = 3, EPL + shear + 10,000 NFW, one
    lens-light and two source Sersic components, 41x41 PSF."""
    r_macro, r_sub, r_ll, r_s1, r_s2, r_psf = _rngs(seed, 6)
    epl, shear = _macro_epl(r_macro)
    nfw = _subhalos(r_sub, n_sub, 1e6, 1e9, 3.0, epl.cx, epl.cy)
    ll = _lens_light(r_ll, epl)
    srcs = [_source(r_s1, 10.0), _source(r_s2, 5.0)]
    grid = Grid(nx=npix, ny=npix, pixel_scale=0.05, supersample=supersample)
    psf = airy_mix_psf(psf_size, 2.0, 3.0, 0.01, r_psf)
    return Scene(grid=grid, lens=Lens(epl=epl, shear=shear, nfw=nfw), source=srcs,
                 lens_light=[ll], psf=psf)


def tnfw_scene(seed: int = 1007, n_sub: int = 10000, npix: int = 200,
               supersample: int = 3, psf_size: int = 41, tau_lo: float = 3.0, tau_hi: float = 30.0) -> Scene:
    """The headline image with truncated subhalos: the same priors, and each
    subhalo truncated at r_trunc = tau Rs with tau log-uniform in
    [tau_lo, tau_hi]; 200x200 px, s = 3, SIE + shear + 10,000 TNFW, one
    lens-light and two source Sersic components, 41x41 PSF."""
    r_macro, r_sub, r_ll, r_s1, r_s2, r_psf, r_tau = _rngs(seed, 7)
    sie, shear = _macro(r_macro)
    nfw = _subhalos(r_sub, n_sub, 1e6, 1e9, 3.0, sie.cx, sie.cy)
    tau = 10.0 ** r_tau.uniform(math.log10(tau_lo), math.log10(tau_hi), size=n_sub)
    nfw.r_trunc = (tau * nfw.Rs.astype(np.float64)).astype(np.float32)
    ll = _lens_light(r_ll, sie)
    srcs = [_source(r_s1, 10.0), _source(r_s2, 5.0)]
    grid = Grid(nx=npix, ny=npix, pixel_scale=0.05, supersample=supersample)
    psf = airy_mix_psf(psf_size, 2.0, 3.0, 0.01, r_psf)
    return Scene(grid=grid, lens=Lens(sie=sie, shear=shear, nfw=nfw), source=srcs,
                 lens_light=[ll], psf=psf)


def config4_scene(seed: int = 1004, n_sub: int = 1000) -> Scene:
    """Differentiation case: 100x100 px at 0.05"/px, no supersampling; the
    plain-method physics plus 1,000 NFW subhalos; 21x21 Gaussian PSF
    (FWHM 0.1", normalised)."""
    r_macro, r_sub, r_src = _rngs(seed, 3)
    sie, shear = _macro(r_macro)
    nfw = _subhalos(r_sub, n_sub, 1e6, 1e9, 3.0, sie.cx, sie.cy)
    src = _source(r_src, 10.0)
    grid = Grid(nx=100, ny=100, pixel_scale=0.05, supersample=1)
    psf = gaussian_psf(21, 0.1 / 0.05)
    return Scene(grid=grid, lens=Lens(sie=sie, shear=shear, nfw=nfw), source=[src], psf=psf)


def config5_scene(seed: int = 1005, n_sub: int = 50000, npix: int = 1000,
                  supersample: int = 5, psf_size: int = 101) -> Scene:
    """Large survey-style case: 1000x1000 px at 0.11"/px, supersampling 5;
    SIE + shear + 50,000 NFW (M log-uniform in [1e6, 1e10], within 6");
    one lens-light + three source Sersic components; 101x101 PSF."""
    r_macro, r_sub, r_ll, r_s1, r_s2, r_s3, r_psf = _rngs(seed, 7)
    sie, shear = _macro(r_macro)
    nfw = _subhalos(r_sub, n_sub, 1e6, 1e10, 6.0, sie.cx, sie.cy)
    ll = _lens_light(r_ll, sie)
    srcs = [_source(r_s1, 10.0), _source(r_s2, 5.0), _source(r_s3, 2.5)]
    grid = Grid(nx=npix, ny=npix, pixel_scale=0.11, supersample=supersample)
    psf = airy_mix_psf(psf_size, 2.0, 3.0, 0.01, r_psf)
    return Scene(grid=grid, lens=Lens(sie=sie, shear=shear, nfw=nfw), source=srcs,
                 lens_light=[ll], psf=psf)


def config3_requests(n_requests: int = 4096, seed: int = 1003, max_sub: int = 20000,
                     sizes=(64, 100, 200, 400), supersamples=(1, 3), psf_sizes=(21, 41)):
    """Serving stream: per request a grid size from `sizes`, a supersampling
    factor from `supersamples`, a log-uniform subhalo count in [0, max_sub] and
    a PSF size from `psf_sizes`; physics as the headline case.  Returns a list
    of Scenes (arrival times are drawn by the caller)."""
    rng_meta, = _rngs(seed, 1)
    out = []
    for i in range(n_requests):
        npx = int(rng_meta.choice(sizes))
        s = int(rng_meta.choice(supersamples))
        nsub = int(math.floor(10.0 ** rng_meta.uniform(0.0, math.log10(max_sub + 1)))) - 1
        k = int(rng_meta.choice(psf_sizes))
        out.append(config2_scene(seed=seed * 100000 + i, n_sub=nsub, npix=npx,
                                 supersample=s, psf_size=k))
    return out


def noisy_image(model, sigma_bkg: float = 0.01, t_exp: float = 1000.0, seed: int = 0):
    """Seeded mock data: Poisson counts of exposure t_exp on max(model, 0),
    divided by t_exp, plus Gaussian background noise sigma_bkg (FP32)."""
    rng = np.random.default_rng(seed)
    m = np.asarray(model, dtype=np.float64)
    d = rng.poisson(t_exp * np.maximum(m, 0.0)) / t_exp + rng.normal(0.0, sigma_bkg, m.shape)
    return d.astype(np.float32)


def config4_draws(B: int = 256, seed: int = 1004, n_sub: int = 1000, grid: Optional[Grid] = None,
                  lens_light: bool = False, psf_size: int = 21):
    """Differentiation case: the truth scene and B parameter draws around it.
    Macro parameters scale by (1 + 0.01 N(0,1)) (q clipped to (0, 1]);
    subhalo x, y move by N(0, 0.005"); alpha_Rs scales by (1 + 0.1 N(0,1))
    (clipped at 0).  Returns (truth, [scene_b])."""
    import copy
    truth = config4_scene(seed=seed, n_sub=n_sub)
    if grid is not None:
        truth.grid = grid
    if psf_size != 21:
        truth.psf = gaussian_psf(psf_size, 0.1 / truth.grid.pixel_scale)
    if lens_light:
        truth.lens_light = [_lens_light(_rngs(seed + 7, 1)[0], truth.lens.sie)]
    rng, = _rngs(seed + 1, 1)
    out = []
    for _ in range(B):
        sc = copy.deepcopy(truth)
        jit = lambda v: f32(v * (1.0 + 0.01 * rng.standard_normal()))
        s = sc.lens.sie
        sc.lens.sie = SIE(jit(s.theta_E), f32(min(1.0, jit(s.q))), jit(s.phi), jit(s.cx), jit(s.cy))
        sc.lens.shear = Shear(jit(sc.lens.shear.gamma1), jit(sc.lens.shear.gamma2))
        sc.source = [Sersic(jit(c.amp), jit(c.R_sersic), jit(c.n_sersic), f32(min(1.0, jit(c.q))), jit(c.phi),
                            jit(c.cx), jit(c.cy)) for c in sc.source]
        sc.lens_light = [Sersic(jit(c.amp), jit(c.R_sersic), jit(c.n_sersic), f32(min(1.0, jit(c.q))),
                                jit(c.phi), jit(c.cx), jit(c.cy)) for c in sc.lens_light]
        n = sc.lens.nfw
        if n is not None and n.n > 0:
            sc.lens.nfw = NFWTable(
                x=(n.x + 0.005 * rng.standard_normal(n.n)).astype(np.float32),
                y=(n.y + 0.005 * rng.standard_normal(n.n)).astype(np.float32),
                Rs=n.Rs.copy(),
                alpha_Rs=np.maximum(n.alpha_Rs * (1.0 + 0.1 * rng.standard_normal(n.n)), 0.0).astype(np.float32))
        out.append(sc)
    return truth, out


def config4_profile_draws(B: int, n_sub: int, grid: Grid, epl: bool, tnfw: bool, seed: int = 1008,
                          psf_size: int = 7):
    """The differentiation case with the other profiles of the deflector
    table: an EPL main deflector (slope 1.9, the SIE's other parameters) in
    place of the SIE and/or truncated subhalos (tau = r_trunc/Rs log-uniform in
    [3, 30]).  Draws jitter the macro parameters (the slope too) by
    (1 + 0.01 N(0,1)) and the subhalos as config4_draws; r_trunc stays fixed.
    Returns (truth, [scene_b])."""
    import copy
    truth, draws = config4_draws(B=B, seed=seed, n_sub=n_sub, grid=grid, psf_size=psf_size)
    rng, = _rngs(seed + 2, 1)
    rt = None
    if tnfw and truth.lens.nfw is not None:
        nfw = truth.lens.nfw
        rt = (10.0 ** rng.uniform(np.log10(3.0), np.log10(30.0), nfw.n) * nfw.Rs).astype(np.float32)
        truth.lens.nfw.r_trunc = rt
    for sc in [truth] + draws:
        if epl:
            s = sc.lens.sie
            g = 1.9 if sc is truth else f32(1.9 * (1.0 + 0.01 * rng.standard_normal()))
            sc.lens.epl = EPL(s.theta_E, g, s.q, s.phi, s.cx, s.cy)
            sc.lens.sie = None
        if rt is not None and sc is not truth:
            sc.lens.nfw = copy.deepcopy(sc.lens.nfw)
            sc.lens.nfw.r_trunc = rt.copy()
    return truth, draws


def random_points(n: int, half_width: float, seed: int):
    """n FP32 points uniform in the square [-half_width, half_width]^2."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(-half_width, half_width, size=(2, n)).astype(np.float32)
    return p[0].copy(), p[1].copy()
