"""Property pins of the oracle's deflections and image steps: invariances that
the lensing formulas must have whatever their parameters (drawn by Hypothesis).

* Translation: moving every deflector centre and every point by the same d
  leaves the deflection unchanged (SIE, EPL, NFW, truncated NFW).
* Rotation: rotating the points, the deflector centres and position angles by
  psi about the origin (and the external shear's (gamma1, gamma2) by 2 psi, a
  spin-2 quantity) rotates the deflection by psi.  A sign slip in a rotation,
  in the shear matrix or in an axis-ratio convention breaks this.
* Superposition and linearity: the deflection of a subhalo set is the sum of
  its parts; NFW, truncated NFW and SIE deflections are linear in alpha_Rs and
  theta_E; the shear's in (gamma1, gamma2) and in the position.
* Image steps: Sersic light is linear in its amplitude and follows its centre;
  the convolution is linear in the image and commutes with a shift of it.
"""
import math

import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

SET = settings(max_examples=25, deadline=None)
REL = 1e-10


def _pts(seed, n=24, half=2.5):
    r = np.random.default_rng(seed)
    return r.uniform(-half, half, n), r.uniform(-half, half, n)


def _close(a, b, rel=REL):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    np.testing.assert_allclose(a, b, rtol=rel, atol=rel * max(np.abs(b).max(), 1e-30))


def _rot(x, y, psi):
    c, s = math.cos(psi), math.sin(psi)
    return c * x - s * y, s * x + c * y


def _subhalos(seed, n, trunc):
    r = np.random.default_rng(seed)
    x, y = r.uniform(-2, 2, n), r.uniform(-2, 2, n)
    rs, ars = r.uniform(0.02, 0.3, n), r.uniform(1e-3, 2e-2, n)
    rt = rs * r.uniform(2.0, 20.0, n) if trunc else None
    return W.NFWTable(x, y, rs, ars, r_trunc=rt)


angles = st.floats(min_value=-math.pi, max_value=math.pi)
shifts = st.floats(min_value=-1.0, max_value=1.0)
seeds = st.integers(min_value=0, max_value=2 ** 31 - 1)
qs = st.floats(min_value=0.2, max_value=0.99)


def _lens_parts(kind, seed, q, phi, gamma=2.0):
    if kind == "sie":
        return W.Lens(sie=W.SIE(1.1, q, phi, 0.07, -0.05))
    if kind == "epl":
        return W.Lens(epl=W.EPL(1.1, gamma, q, phi, 0.07, -0.05))
    return W.Lens(nfw=_subhalos(seed, 5, kind == "tnfw"))


def _moved(lens, f):
    """lens with every centre (x, y) -> f(x, y) and position angle phi -> phi + dphi."""
    out = W.Lens()
    fx, dphi = f
    if lens.sie is not None:
        s = lens.sie
        cx, cy = fx(s.cx, s.cy)
        out.sie = W.SIE(s.theta_E, s.q, s.phi + dphi, float(cx), float(cy))
    if lens.epl is not None:
        e = lens.epl
        cx, cy = fx(e.cx, e.cy)
        out.epl = W.EPL(e.theta_E, e.gamma, e.q, e.phi + dphi, float(cx), float(cy))
    if lens.nfw is not None:
        n = lens.nfw
        x, y = fx(n.x, n.y)
        out.nfw = W.NFWTable(np.asarray(x), np.asarray(y), n.Rs, n.alpha_Rs, r_trunc=n.r_trunc)
    return out


@pytest.mark.parametrize("kind", ["sie", "epl", "nfw", "tnfw"])
@SET
@given(seed=seeds, dx=shifts, dy=shifts, q=qs, phi=angles, gamma=st.floats(min_value=1.3, max_value=2.7))
def test_translation(kind, seed, dx, dy, q, phi, gamma):
    lens = _lens_parts(kind, seed, q, phi, gamma)
    x, y = _pts(seed)
    a = O.total_deflection(x, y, lens)
    moved = _moved(lens, (lambda u, v: (u + dx, v + dy), 0.0))
    b = O.total_deflection(x + dx, y + dy, moved)
    _close(b[0], a[0])
    _close(b[1], a[1])


@pytest.mark.parametrize("kind", ["sie", "epl", "nfw", "tnfw"])
@SET
@given(seed=seeds, psi=angles, q=qs, phi=angles, gamma=st.floats(min_value=1.3, max_value=2.7))
def test_rotation(kind, seed, psi, q, phi, gamma):
    lens = _lens_parts(kind, seed, q, phi, gamma)
    x, y = _pts(seed)
    ax, ay = O.total_deflection(x, y, lens)
    rotated = _moved(lens, (lambda u, v: _rot(u, v, psi), psi))
    xr, yr = _rot(x, y, psi)
    bx, by = O.total_deflection(xr, yr, rotated)
    ex, ey = _rot(ax, ay, psi)
    _close(bx, ex)
    _close(by, ey)


@SET
@given(seed=seeds, psi=angles, g1=st.floats(-0.1, 0.1), g2=st.floats(-0.1, 0.1))
def test_shear_is_spin_two(seed, psi, g1, g2):
    x, y = _pts(seed)
    ax, ay = O.shear_deflection(x, y, g1, g2)
    c2, s2 = math.cos(2 * psi), math.sin(2 * psi)
    xr, yr = _rot(x, y, psi)
    bx, by = O.shear_deflection(xr, yr, g1 * c2 - g2 * s2, g1 * s2 + g2 * c2)
    ex, ey = _rot(ax, ay, psi)
    _close(bx, ex)
    _close(by, ey)


@SET
@given(seed=seeds, a=st.floats(0.1, 3.0), b=st.floats(-2.0, 2.0), g1=st.floats(-0.1, 0.1),
       g2=st.floats(-0.1, 0.1), h1=st.floats(-0.1, 0.1), h2=st.floats(-0.1, 0.1))
def test_shear_is_linear(seed, a, b, g1, g2, h1, h2):
    x, y = _pts(seed)
    u, v = _pts(seed + 1)
    s = O.shear_deflection(a * x + b * u, a * y + b * v, g1, g2)
    p = O.shear_deflection(x, y, g1, g2)
    q = O.shear_deflection(u, v, g1, g2)
    _close(s[0], a * p[0] + b * q[0], 1e-12)
    _close(s[1], a * p[1] + b * q[1], 1e-12)
    t = O.shear_deflection(x, y, g1 + h1, g2 + h2)
    r = O.shear_deflection(x, y, h1, h2)
    _close(t[0], p[0] + r[0], 1e-12)
    _close(t[1], p[1] + r[1], 1e-12)


@pytest.mark.parametrize("trunc", [False, True])
@SET
@given(seed=seeds, k=st.integers(1, 6), scale=st.floats(0.1, 10.0))
def test_subhalo_superposition_and_amplitude(trunc, seed, k, scale):
    n = _subhalos(seed, 7, trunc)
    x, y = _pts(seed)
    whole = O.total_deflection(x, y, W.Lens(nfw=n))

    def part(sl):
        return W.NFWTable(n.x[sl], n.y[sl], n.Rs[sl], n.alpha_Rs[sl],
                          r_trunc=None if n.r_trunc is None else n.r_trunc[sl])
    a = O.total_deflection(x, y, W.Lens(nfw=part(slice(0, k))))
    b = O.total_deflection(x, y, W.Lens(nfw=part(slice(k, None))))
    _close(whole[0], a[0] + b[0])
    _close(whole[1], a[1] + b[1])
    scaled = W.NFWTable(n.x, n.y, n.Rs, scale * n.alpha_Rs, r_trunc=n.r_trunc)
    s = O.total_deflection(x, y, W.Lens(nfw=scaled))
    _close(s[0], scale * whole[0])
    _close(s[1], scale * whole[1])


@SET
@given(seed=seeds, q=qs, phi=angles, scale=st.floats(0.1, 10.0))
def test_sie_is_linear_in_theta_E(seed, q, phi, scale):
    x, y = _pts(seed)
    a = O.sie_deflection(x, y, 1.1, q, phi, 0.07, -0.05)
    b = O.sie_deflection(x, y, 1.1 * scale, q, phi, 0.07, -0.05)
    _close(b[0], scale * a[0])
    _close(b[1], scale * a[1])


@SET
@given(seed=seeds, amp=st.floats(0.1, 50.0), dx=shifts, dy=shifts, n=st.floats(0.6, 6.0), q=qs, phi=angles)
def test_sersic_linear_and_follows_its_centre(seed, amp, dx, dy, n, q, phi):
    x, y = _pts(seed)
    base = O.sersic(x, y, 1.0, 0.3, n, q, phi, 0.1, -0.2)
    _close(O.sersic(x, y, amp, 0.3, n, q, phi, 0.1, -0.2), amp * base)
    _close(O.sersic(x + dx, y + dy, 1.0, 0.3, n, q, phi, 0.1 + dx, -0.2 + dy), base)
    # and it is the surface brightness of a lone source component at beta
    sb = O.surface_brightness(x, y, x, y, [W.Sersic(amp, 0.3, n, q, phi, 0.1, -0.2)], [], bn_exact=False)
    _close(sb, amp * base)


@SET
@given(seed=seeds, a=st.floats(-3.0, 3.0), b=st.floats(-3.0, 3.0), k=st.sampled_from([1, 3, 5, 7]),
       sx=st.integers(-3, 3), sy=st.integers(-3, 3))
def test_convolution_linear_and_shift_equivariant(seed, a, b, k, sx, sy):
    r = np.random.default_rng(seed)
    n = 24
    f, g = r.uniform(-1, 1, (n, n)), r.uniform(-1, 1, (n, n))
    ker = r.uniform(0, 1, (k, k))
    lin = O.convolve_same(a * f + b * g, ker)
    _close(lin, a * O.convolve_same(f, ker) + b * O.convolve_same(g, ker), 1e-12)
    # an image that is zero near its border, shifted inside the frame
    h = np.zeros((n, n))
    h[8:16, 8:16] = r.uniform(0, 1, (8, 8))
    hs = np.roll(np.roll(h, sy, axis=0), sx, axis=1)
    c0 = O.convolve_same(h, ker)
    c1 = O.convolve_same(hs, ker)
    _close(c1, np.roll(np.roll(c0, sy, axis=0), sx, axis=1), 1e-12)
