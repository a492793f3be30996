"""Pins of the oracle's grid, Sersic light, convolution and composed
simulation against closed forms, library routines and invariants.

* Grid: hand-computed sub-pixel centres; the sub-pixel mean of a linear
  function is its value at the pixel centre.
* Sersic: I(R_sersic) = amp; total flux 2 pi n R^2 amp e^b b^(-2n) Gamma(2n)
  (independent of q) from a 2-D sum over a fine grid; half-light radius under
  the exact b_n; the exact b_n through scipy's incomplete-gamma inverse.
* Convolution: scipy.signal.convolve2d(mode='same') with an asymmetric kernel;
  delta PSF = identity; unit-sum kernel conserves flux.
* Composition: SIS + centred circular source gives I(theta) = S(| |theta| - theta_E |);
  the Einstein ring peaks at theta_E; with no lens the image sums to the total flux.
"""
import math

import numpy as np
import pytest
from scipy.signal import convolve2d
from scipy.special import gamma, gammainc

import oracle as O
import workloads as W


# ---------------------------------------------------------------- grid
def test_grid_hand_values():
    tx, ty = O.subpixel_coords(2, 1, 1.0, 0.0, 0.0, 1)
    np.testing.assert_array_equal(tx.reshape(-1), [-0.5, 0.5])
    np.testing.assert_array_equal(ty.reshape(-1), [0.0, 0.0])
    tx, ty = O.subpixel_coords(2, 3, 0.5, 1.0, -2.0, 2)
    # pixel (row 0, col 0): centre (0.75, -2.5); sub-pixels at +-0.125
    np.testing.assert_allclose(tx[0, 0], [[0.625, 0.875], [0.625, 0.875]])
    np.testing.assert_allclose(ty[0, 0], [[-2.625, -2.625], [-2.375, -2.375]])
    np.testing.assert_allclose(ty[2, 1, 1, 1], -2.0 + 0.5 + 0.125)


@pytest.mark.parametrize("s", [1, 2, 3, 5])
def test_grid_linear_mean_is_pixel_centre(s):
    d = 0.05
    tx, ty = O.subpixel_coords(7, 4, d, 0.3, -0.1, s)
    lin = 2.0 * tx - 3.0 * ty + 1.0
    px = O.supersample_reduce(lin, d) / d ** 2
    cx = 0.3 + (np.arange(7) - 3.0) * d
    cy = -0.1 + (np.arange(4) - 1.5) * d
    np.testing.assert_allclose(px, 2 * cx[None, :] - 3 * cy[:, None] + 1.0, atol=1e-13)
    # constant SB -> pixel = area * SB
    np.testing.assert_allclose(O.supersample_reduce(np.full(tx.shape, 4.0), d), 4.0 * d * d)


# ---------------------------------------------------------------- Sersic
def _total_flux(amp, R, n, b):
    return 2 * math.pi * n * R * R * amp * math.exp(b) * b ** (-2 * n) * gamma(2 * n)


def test_sersic_amp_at_R_sersic():
    amp, R, n, q, phi = 7.0, 0.3, 2.5, 0.7, 0.9
    for ang in (0.0, 1.0, 2.5):
        # point on the isophote R = R_sersic: x' = R cos(t)/sqrt(q), y' = R sqrt(q) sin(t)
        xp, yp = R * math.cos(ang) / math.sqrt(q), R * math.sqrt(q) * math.sin(ang)
        c, s = math.cos(phi), math.sin(phi)
        x, y = 0.1 + c * xp - s * yp, -0.2 + s * xp + c * yp
        v = O.sersic(np.array([x]), np.array([y]), amp, R, n, q, phi, 0.1, -0.2)[0]
        assert abs(v - amp) < 1e-13 * amp


@pytest.mark.parametrize("n,q", [(1.0, 1.0), (2.0, 0.6), (3.5, 0.85)])
def test_sersic_total_flux_on_fine_grid(n, q):
    amp, R, phi = 3.0, 0.25, 0.4
    d = 0.004
    half = 40 * R if n > 3 else 25 * R
    ax = np.arange(-half, half, d) + d / 2      # cell centres; the cusp sits on a cell corner
    x, y = np.meshgrid(ax, ax)
    img = O.sersic(x, y, amp, R, n, q, phi, 0.0, 0.0)
    flux = img.sum() * d * d
    b = O.sersic_bn(n)
    expect = _total_flux(amp, R, n, b)
    # midpoint-rule error plus the flux beyond the box stay below 1e-3 here;
    # a wrong elliptical radius would be off by a factor of q^(+-1/2) or q^(+-1)
    assert abs(flux - expect) < 1.5e-3 * expect


@pytest.mark.parametrize("n", [0.8, 1.0, 2.0, 4.0])
def test_sersic_half_light_radius_with_exact_bn(n):
    b = O.sersic_bn(n, exact=True)
    assert abs(gammainc(2 * n, b) - 0.5) < 1e-12
    # numeric check of the flux inside R_sersic from the profile itself (q = 1, radial integral)
    from scipy.integrate import quad
    R = 0.3
    prof = lambda r: O.sersic(np.array([r]), np.array([0.0]), 1.0, R, n, 1.0, 0.0, 0.0, 0.0, True)[0] * 2 * math.pi * r
    inner, _ = quad(prof, 0, R, epsrel=1e-11, limit=200)
    total = _total_flux(1.0, R, n, b)
    assert abs(inner / total - 0.5) < 1e-8


def test_sersic_bn_linear_fit_close_to_exact():
    # Capaccioli's linear fit differs from the exact value by ~6e-3 at n = 1
    assert abs(O.sersic_bn(1.0) - O.sersic_bn(1.0, exact=True)) < 1e-2
    assert O.sersic_bn(4.0) == pytest.approx(1.9992 * 4 - 0.3271)


def test_sersic_centre_and_circular_rotation_invariance():
    v0 = O.sersic(np.array([0.5]), np.array([0.5]), 2.0, 0.2, 3.0, 0.8, 0.3, 0.5, 0.5)[0]
    assert v0 == pytest.approx(2.0 * math.exp(O.sersic_bn(3.0)), rel=1e-14)
    rng = np.random.default_rng(4)
    x, y = rng.uniform(-1, 1, (2, 30))
    a = O.sersic(x, y, 1.0, 0.3, 2.0, 1.0, 0.0, 0.0, 0.0)
    b = O.sersic(x, y, 1.0, 0.3, 2.0, 1.0, 1.234, 0.0, 0.0)
    np.testing.assert_allclose(a, b, rtol=1e-13)


# ---------------------------------------------------------------- convolution
@pytest.mark.parametrize("k,shape", [(1, (5, 7)), (3, (9, 6)), (7, (20, 31)), (11, (8, 8)), (15, (6, 9))])
def test_convolution_matches_scipy(k, shape):
    rng = np.random.default_rng(k)
    img = rng.standard_normal(shape)
    K = rng.uniform(0, 1, (k, k))
    K[0, :] *= 3.0                        # asymmetric: a flipped kernel would differ
    out = O.convolve_same(img, K)
    ref = convolve2d(img, K, mode="same", boundary="fill", fillvalue=0.0)
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("k,shape", [(3, (9, 6)), (11, (8, 8)), (15, (6, 9)), (21, (40, 13))])
def test_sampled_convolution_matches_scipy(k, shape):
    rng = np.random.default_rng(k + 100)
    img = rng.standard_normal(shape)
    K = rng.uniform(0, 1, (k, k))
    K[:, 0] *= 5.0
    ref = convolve2d(img, K, mode="same", boundary="fill", fillvalue=0.0)
    rows, cols = np.divmod(np.arange(img.size), shape[1])
    np.testing.assert_allclose(O.convolve_at(img, K, rows, cols), ref.ravel(), rtol=1e-12, atol=1e-12)


def test_convolution_delta_and_flux():
    rng = np.random.default_rng(0)
    img = rng.uniform(0, 1, (30, 40))
    delta = np.zeros((9, 9))
    delta[4, 4] = 1.0
    np.testing.assert_array_equal(O.convolve_same(img, delta), img)
    K = W.gaussian_psf(9, 2.0).astype(np.float64)
    K /= K.sum()
    core = np.zeros((30, 40))
    core[8:22, 8:32] = img[8:22, 8:32]     # support >= c px from the edge
    np.testing.assert_allclose(O.convolve_same(core, K).sum(), core.sum(), rtol=1e-13)
    # a single off-centre tap shifts the image: K[a, b] at (c+1, c) moves rows down by 1
    shift = np.zeros((3, 3))
    shift[2, 1] = 1.0
    out = O.convolve_same(img, shift)
    np.testing.assert_array_equal(out[1:], img[:-1])
    np.testing.assert_array_equal(out[0], 0.0)


# ---------------------------------------------------------------- composition
def _scene(lens, source, nx=60, d=0.05, s=1):
    return W.Scene(grid=W.Grid(nx=nx, ny=nx, pixel_scale=d, supersample=s), lens=lens,
                   source=source, lens_light=[], psf=None)


def test_sis_with_centred_source_maps_radius():
    te = 1.0
    src = W.Sersic(amp=2.0, R_sersic=0.2, n_sersic=1.5, q=1.0, phi=0.0, cx=0.0, cy=0.0)
    scene = _scene(W.Lens(sie=W.SIE(te, 1.0, 0.0, 0.0, 0.0)), [src])
    img = O.simulate_unconvolved(scene)
    tx, ty = O.subpixel_coords(60, 60, 0.05, 0.0, 0.0, 1)
    rad = np.abs(np.hypot(tx, ty) - te)[..., 0, 0]
    b = O.sersic_bn(1.5)
    expect = 0.05 ** 2 * 2.0 * np.exp(-b * ((rad / 0.2) ** (1 / 1.5) - 1))
    np.testing.assert_allclose(img, expect, rtol=1e-12)


def test_einstein_ring_peaks_at_theta_E():
    te = 0.9
    src = W.Sersic(amp=1.0, R_sersic=0.05, n_sersic=1.0, q=1.0, phi=0.0, cx=0.0, cy=0.0)
    scene = _scene(W.Lens(sie=W.SIE(te, 1.0, 0.0, 0.0, 0.0)), [src], nx=120, d=0.025)
    img = O.simulate_unconvolved(scene)
    tx, ty = O.subpixel_coords(120, 120, 0.025, 0.0, 0.0, 1)
    r = np.hypot(tx, ty)[..., 0, 0]
    bins = np.arange(0.0, 1.5, 0.025)
    prof = [img[(r >= lo) & (r < lo + 0.025)].mean() for lo in bins]
    peak = bins[int(np.argmax(prof))] + 0.0125
    assert abs(peak - te) <= 0.025


def test_unlensed_image_sums_to_total_flux():
    src = W.Sersic(amp=1.5, R_sersic=0.3, n_sersic=1.0, q=0.7, phi=0.5, cx=0.02, cy=-0.01)
    scene = _scene(W.Lens(), [src], nx=400, d=0.02, s=3)
    flux = O.simulate_unconvolved(scene).sum()
    expect = _total_flux(1.5, 0.3, 1.0, O.sersic_bn(1.0))
    assert abs(flux - expect) < 1e-6 * expect


def test_simulate_convolution_conserves_and_lens_light_unlensed():
    sc = W.config1_scene(draw=3)
    sc.lens_light = [W.Sersic(amp=1.0, R_sersic=0.5, n_sersic=2.0, q=0.9, phi=0.1, cx=0.0, cy=0.0)]
    un = O.simulate_unconvolved(sc)
    full = O.simulate_image(sc)
    np.testing.assert_allclose(full, O.convolve_same(un, sc.psf), rtol=1e-14)
    # lens light part: evaluated at theta, independent of the lens
    sc2 = W.Scene(grid=sc.grid, lens=W.Lens(), source=[], lens_light=sc.lens_light, psf=None)
    sc3 = W.Scene(grid=sc.grid, lens=sc.lens, source=[], lens_light=sc.lens_light, psf=None)
    np.testing.assert_allclose(O.simulate_unconvolved(sc2), O.simulate_unconvolved(sc3), rtol=1e-15)
