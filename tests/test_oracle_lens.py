"""Pins of the oracle's deflection profiles against closed forms, invariants,
quadrature and high-precision arithmetic -- nothing here re-types the oracle's
own deflection formulas.

* SIS: |alpha| = theta_E everywhere (Einstein-radius definition).
* SIE: Schramm's one-dimensional integral for homoeoidal mass distributions
  (Keeton 2001 catalogue) evaluated by quadrature from the convergence alone;
  div alpha = 2 kappa and curl alpha = 0 by central differences; continuity of
  the q -> 1 series branch.
* EPL: the same homoeoid integral for the power-law convergence; the circular
  case |alpha| = theta_E^(gamma-1) r^(2-gamma); div alpha = 2 kappa, curl
  alpha = 0; gamma = 2 is the SIE.
* Shear: the complex form alpha = gamma * conj(z) and its constant Hessian.
* NFW: kappa against a numerical line-of-sight projection of the 3-D NFW
  density; alpha against the enclosed-mass integral of kappa; 50-digit mpmath
  values of g(x); |alpha(Rs)| = alpha_Rs; div alpha = 2 kappa; linearity.
* TNFW: alpha against the mass of the truncated 3-D density inside the
  cylinder of radius r (one-dimensional quadrature over spherical shells); the
  untruncated limit is the NFW; the far-field limit is the total mass of the
  density; zero at the centre, linear in alpha_Rs.
* Point mass: the two image positions of the quadratic lens equation.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.integrate import quad

import oracle as O


def _div_curl(fun, x, y, h):
    axp, _ = fun(x + h, y)
    axm, _ = fun(x - h, y)
    _, ayp = fun(x, y + h)
    _, aym = fun(x, y - h)
    div = (axp - axm) / (2 * h) + (ayp - aym) / (2 * h)
    _, ay_xp = fun(x + h, y)
    _, ay_xm = fun(x - h, y)
    ax_yp, _ = fun(x, y + h)
    ax_ym, _ = fun(x, y - h)
    curl = (ay_xp - ay_xm) / (2 * h) - (ax_yp - ax_ym) / (2 * h)
    return div, curl


# ---------------------------------------------------------------- SIS / SIE
def test_sis_modulus_is_theta_E():
    rng = np.random.default_rng(0)
    x, y = rng.uniform(-3, 3, (2, 500))
    ax, ay = O.sie_deflection(x, y, 1.2, 1.0, 0.3, 0.1, -0.2)
    np.testing.assert_allclose(np.hypot(ax, ay), 1.2, rtol=1e-14)
    # radial direction
    np.testing.assert_allclose(ax * (y + 0.2) - ay * (x - 0.1), 0.0, atol=1e-13)


def test_sie_centre_is_zero():
    ax, ay = O.sie_deflection(np.array([0.25]), np.array([-0.5]), 1.0, 0.7, 0.4, 0.25, -0.5)
    assert ax[0] == 0.0 and ay[0] == 0.0


def _schramm(xp, yp, theta_E, q):
    """alpha in the major-axis frame from the convergence of an SIE alone:
    kappa(xi) = theta_E / (2 sqrt(q) xi), xi^2 = x^2 + y^2/q^2, via
    alpha_x = q x J0, alpha_y = q y J1,
    J_n = int_0^1 kappa(xi(u)^2) / (1 - (1-q^2) u)^(n+1/2) du,
    xi(u)^2 = u (x^2 + y^2 / (1 - (1-q^2) u))."""
    e = 1.0 - q * q

    def h(u, n):
        d = 1.0 - e * u
        # kappa(xi(u)) = theta_E/(2 sqrt q) * u^-1/2 * (x^2 + y^2/d)^-1/2 ; u^-1/2 via weight
        return theta_E / (2.0 * math.sqrt(q)) / math.sqrt(xp * xp + yp * yp / d) / d ** (n + 0.5)

    j0, _ = quad(h, 0.0, 1.0, args=(0,), weight="alg", wvar=(-0.5, 0.0), epsabs=1e-14, epsrel=1e-13)
    j1, _ = quad(h, 0.0, 1.0, args=(1,), weight="alg", wvar=(-0.5, 0.0), epsabs=1e-14, epsrel=1e-13)
    return q * xp * j0, q * yp * j1


@pytest.mark.parametrize("q", [0.55, 0.8, 0.97])
def test_sie_matches_homoeoid_quadrature(q):
    theta_E, phi, cx, cy = 1.1, 0.7, 0.05, -0.03
    rng = np.random.default_rng(int(q * 100))
    pts = rng.uniform(-2.5, 2.5, (12, 2))
    c, s = math.cos(phi), math.sin(phi)
    for px, py in pts:
        ax, ay = O.sie_deflection(np.array([px]), np.array([py]), theta_E, q, phi, cx, cy)
        dx, dy = px - cx, py - cy
        xp, yp = c * dx + s * dy, -s * dx + c * dy
        axp, ayp = _schramm(xp, yp, theta_E, q)
        ex, ey = c * axp - s * ayp, s * axp + c * ayp
        assert abs(ax[0] - ex) < 1e-9 and abs(ay[0] - ey) < 1e-9


@pytest.mark.parametrize("q", [0.6, 0.85, 1.0 - 1e-8])
def test_sie_divergence_and_curl(q):
    theta_E, phi, cx, cy = 1.3, 2.1, -0.04, 0.02
    rng = np.random.default_rng(7)
    x, y = rng.uniform(-2, 2, (2, 60))
    fun = lambda a, b: O.sie_deflection(a, b, theta_E, q, phi, cx, cy)
    div, curl = _div_curl(fun, x, y, 1e-5)
    kap = O.sie_kappa(x, y, theta_E, q, phi, cx, cy)
    np.testing.assert_allclose(div, 2 * kap, rtol=2e-7)
    assert np.max(np.abs(curl)) < 1e-6


def test_sie_series_branch_is_continuous():
    rng = np.random.default_rng(3)
    x, y = rng.uniform(-2, 2, (2, 100))
    a_sis = O.sie_deflection(x, y, 1.0, 1.0, 0.2, 0.0, 0.0)
    a_ser = O.sie_deflection(x, y, 1.0, 1.0 - 1e-7, 0.2, 0.0, 0.0)     # f ~ 4.5e-4: series
    a_dir = O.sie_deflection(x, y, 1.0, 1.0 - 1e-6, 0.2, 0.0, 0.0)     # f ~ 1.4e-3: atan/atanh
    np.testing.assert_allclose(a_ser[0], a_sis[0], atol=2e-7)
    np.testing.assert_allclose(a_dir[0], a_ser[0], atol=2e-6)
    np.testing.assert_allclose(a_dir[1], a_ser[1], atol=2e-6)


# ---------------------------------------------------------------- EPL
def _schramm_power_law(xp, yp, theta_E, gamma, q):
    """alpha in the major-axis frame of the homoeoidal convergence
    kappa(xi) = (3 - gamma)/2 * (theta_E / (sqrt(q) xi))^(gamma - 1),
    xi^2 = x^2 + y^2/q^2, by the same one-dimensional integrals as
    `_schramm`: along the path kappa(xi(u)) carries u^(-(gamma-1)/2), taken as
    the quadrature weight."""
    e = 1.0 - q * q
    p = gamma - 1.0

    def h(u, n):
        d = 1.0 - e * u
        return (0.5 * (3.0 - gamma) * (theta_E / math.sqrt(q)) ** p
                * (xp * xp + yp * yp / d) ** (-0.5 * p) / d ** (n + 0.5))

    j0, _ = quad(h, 0.0, 1.0, args=(0,), weight="alg", wvar=(-0.5 * p, 0.0), epsabs=1e-14, epsrel=1e-13)
    j1, _ = quad(h, 0.0, 1.0, args=(1,), weight="alg", wvar=(-0.5 * p, 0.0), epsabs=1e-14, epsrel=1e-13)
    return q * xp * j0, q * yp * j1


@pytest.mark.parametrize("gamma,q", [(1.5, 0.5), (2.0, 0.7), (2.4, 0.85), (1.8, 0.3), (1.9, 0.05)])
def test_epl_matches_homoeoid_quadrature(gamma, q):
    theta_E, phi, cx, cy = 1.05, 0.9, -0.06, 0.04
    rng = np.random.default_rng(int(gamma * 10 + q * 100))
    pts = rng.uniform(-2.5, 2.5, (10, 2))
    c, s = math.cos(phi), math.sin(phi)
    for px, py in pts:
        ax, ay = O.epl_deflection(np.array([px]), np.array([py]), theta_E, gamma, q, phi, cx, cy)
        dx, dy = px - cx, py - cy
        xp, yp = c * dx + s * dy, -s * dx + c * dy
        axp, ayp = _schramm_power_law(xp, yp, theta_E, gamma, q)
        ex, ey = c * axp - s * ayp, s * axp + c * ayp
        assert abs(ax[0] - ex) < 1e-9 * max(1.0, abs(ex)) and abs(ay[0] - ey) < 1e-9 * max(1.0, abs(ey))


@pytest.mark.parametrize("gamma", [1.3, 2.0, 2.7])
def test_epl_circular_is_power_law(gamma):
    rng = np.random.default_rng(11)
    x, y = rng.uniform(-3, 3, (2, 300))
    ax, ay = O.epl_deflection(x, y, 0.9, gamma, 1.0, 0.4, 0.1, -0.2)
    r = np.hypot(x - 0.1, y + 0.2)
    np.testing.assert_allclose(np.hypot(ax, ay), 0.9 ** (gamma - 1.0) * r ** (2.0 - gamma), rtol=1e-13)
    np.testing.assert_allclose(ax * (y + 0.2) - ay * (x - 0.1), 0.0, atol=1e-12)


@pytest.mark.parametrize("gamma,q", [(1.6, 0.4), (2.3, 0.75), (1.2, 0.2)])
def test_epl_divergence_and_curl(gamma, q):
    theta_E, phi, cx, cy = 1.1, 0.7, 0.2, 0.1
    rng = np.random.default_rng(5)
    x, y = rng.uniform(-2, 2, (2, 80))
    keep = np.hypot(x - cx, y - cy) > 0.2
    x, y = x[keep], y[keep]
    fun = lambda a, b: O.epl_deflection(a, b, theta_E, gamma, q, phi, cx, cy)
    div, curl = _div_curl(fun, x, y, 1e-5)
    kap = O.epl_kappa(x, y, theta_E, gamma, q, phi, cx, cy)
    np.testing.assert_allclose(div, 2 * kap, rtol=1e-7)
    assert np.max(np.abs(curl) / kap) < 1e-6


def test_epl_gamma_two_is_sie_and_centre_is_zero():
    rng = np.random.default_rng(2)
    x, y = rng.uniform(-2, 2, (2, 100))
    for q in (0.45, 0.9, 1.0):
        a = O.epl_deflection(x, y, 1.2, 2.0, q, 0.4, 0.1, -0.05)
        b = O.sie_deflection(x, y, 1.2, q, 0.4, 0.1, -0.05)
        np.testing.assert_allclose(a[0], b[0], atol=1e-13)
        np.testing.assert_allclose(a[1], b[1], atol=1e-13)
    ax, ay = O.epl_deflection(np.array([0.1]), np.array([-0.05]), 1.2, 2.5, 0.6, 0.4, 0.1, -0.05)
    assert ax[0] == 0.0 and ay[0] == 0.0
    ax, ay = O.epl_deflection(x, y, 0.0, 1.5, 0.6, 0.4, 0.1, -0.05)
    assert not np.any(ax) and not np.any(ay)


# ---------------------------------------------------------------- shear
def test_shear_complex_form_and_hessian():
    rng = np.random.default_rng(1)
    x, y = rng.uniform(-2, 2, (2, 50))
    g1, g2 = 0.031, -0.017
    ax, ay = O.shear_deflection(x, y, g1, g2)
    z = (g1 + 1j * g2) * np.conj(x + 1j * y)
    np.testing.assert_allclose(ax, z.real, atol=1e-15)
    np.testing.assert_allclose(ay, z.imag, atol=1e-15)
    div, curl = _div_curl(lambda a, b: O.shear_deflection(a, b, g1, g2), x, y, 1e-3)
    np.testing.assert_allclose(div, 0.0, atol=1e-12)
    np.testing.assert_allclose(curl, 0.0, atol=1e-12)


# ---------------------------------------------------------------- NFW
def _kappa_projected(X, kappa_s):
    """kappa(x) = 2 kappa_s int_0^inf dz / (s (1+s)^2), s = sqrt(x^2+z^2):
    the 3-D NFW profile rho_s / ((r/rs)(1+r/rs)^2) projected along the line of
    sight, in units of rho_s rs / Sigma_crit = kappa_s."""
    f = lambda z: 1.0 / (math.sqrt(X * X + z * z) * (1.0 + math.sqrt(X * X + z * z)) ** 2)
    v1, _ = quad(f, 0.0, 1.0, epsabs=0, epsrel=1e-12, limit=200)
    v2, _ = quad(f, 1.0, np.inf, epsabs=0, epsrel=1e-12, limit=200)
    return 2.0 * kappa_s * (v1 + v2)


@pytest.mark.parametrize("X", [0.01, 0.3, 0.9, 0.99, 1.0, 1.01, 1.2, 3.0, 40.0])
def test_nfw_kappa_is_projected_density(X):
    Rs, aRs = 0.2, 3e-3
    ks = aRs / (4 * Rs * (1 - math.log(2)))
    k = O.nfw_kappa(np.array([X * Rs]), np.array([0.0]), Rs, aRs, 0.0, 0.0)[0]
    assert abs(k - _kappa_projected(X, ks)) <= 1e-9 * abs(k)


@pytest.mark.parametrize("X", [0.02, 0.5, 0.95, 1.0, 1.05, 2.0, 10.0, 300.0])
def test_nfw_alpha_is_enclosed_mass(X):
    Rs, aRs = 0.15, 2e-3
    r = X * Rs
    ax, ay = O.nfw_deflection(np.array([r]), np.array([0.0]), Rs, aRs, 0.0, 0.0)
    kap = lambda rr: O.nfw_kappa(np.array([rr]), np.array([0.0]), Rs, aRs, 0.0, 0.0)[0] * rr
    pts = [p * Rs for p in (0.5, 1.0, 2.0) if p * Rs < r]
    m, _ = quad(kap, 0.0, r, points=pts or None, epsabs=0, epsrel=1e-12, limit=400)
    expect = 2.0 * m / r
    assert abs(ax[0] - expect) <= 1e-9 * expect
    assert ay[0] == 0.0


def test_nfw_alpha_at_Rs_is_alpha_Rs():
    rng = np.random.default_rng(5)
    ang = rng.uniform(0, 2 * np.pi, 20)
    Rs, aRs, cx, cy = 0.07, 1.3e-3, 0.4, -0.9
    ax, ay = O.nfw_deflection(cx + Rs * np.cos(ang), cy + Rs * np.sin(ang), Rs, aRs, cx, cy)
    np.testing.assert_allclose(np.hypot(ax, ay), aRs, rtol=1e-14)


@pytest.mark.parametrize("X", ["1e-6", "1e-3", "0.3", "0.5", "0.9", "0.999999", "1",
                               "1.000001", "1.1", "2", "1e3"])
def test_nfw_g_against_mpmath(X):
    mp.mp.dps = 50
    x = mp.mpf(X)
    if x < 1:
        F = mp.acosh(1 / x) / mp.sqrt(1 - x * x)
    elif x > 1:
        F = mp.acos(1 / x) / mp.sqrt(x * x - 1)
    else:
        F = mp.mpf(1)
    g_ref = mp.log(x / 2) + F
    g = O.nfw_g(np.array([float(x)]))[0]
    assert abs(g - float(g_ref)) <= 4e-15 * abs(float(g_ref)) + 1e-300


def test_nfw_divergence_is_twice_kappa():
    Rs, aRs, cx, cy = 0.1, 2e-3, 0.01, -0.02
    ang = np.linspace(0.1, 6.0, 7)
    for X in (0.2, 0.7, 0.97, 1.0, 1.04, 1.6, 8.0):
        x = cx + X * Rs * np.cos(ang)
        y = cy + X * Rs * np.sin(ang)
        div, curl = _div_curl(lambda a, b: O.nfw_deflection(a, b, Rs, aRs, cx, cy), x, y, 1e-6 * Rs)
        kap = O.nfw_kappa(x, y, Rs, aRs, cx, cy)
        np.testing.assert_allclose(div, 2 * kap, rtol=3e-6)
        assert np.max(np.abs(curl)) < 3e-6 * np.max(kap)


def test_nfw_linear_in_alpha_Rs_and_superposes():
    rng = np.random.default_rng(11)
    x, y = rng.uniform(-1, 1, (2, 40))
    Rs = np.array([0.05, 0.2, 0.1])
    aRs = np.array([1e-3, 4e-3, 2e-4])
    cx = np.array([0.1, -0.3, 0.5])
    cy = np.array([0.0, 0.2, -0.4])
    ax, ay = O.nfw_deflection(x, y, Rs, aRs, cx, cy)
    sx = sum(O.nfw_deflection(x, y, Rs[k], aRs[k], cx[k], cy[k])[0] for k in range(3))
    np.testing.assert_allclose(ax, sx, rtol=1e-13, atol=1e-18)
    ax2, _ = O.nfw_deflection(x, y, Rs, 3 * aRs, cx, cy)
    np.testing.assert_allclose(ax2, 3 * ax, rtol=1e-13)


def test_nfw_zero_at_centre_and_chunking_invariant():
    Rs, aRs = np.array([0.1, 0.2]), np.array([1e-3, 2e-3])
    cx, cy = np.array([0.3, -0.1]), np.array([0.2, 0.4])
    ax, ay = O.nfw_deflection(np.array([0.3]), np.array([0.2]), Rs[:1], aRs[:1], cx[:1], cy[:1])
    assert ax[0] == 0.0 and ay[0] == 0.0
    rng = np.random.default_rng(2)
    x, y = rng.uniform(-1, 1, (2, 37))
    a1 = O.nfw_deflection(x, y, Rs, aRs, cx, cy)
    a2 = O.nfw_deflection(x, y, Rs, aRs, cx, cy, chunk_points=5, chunk_sub=1)
    np.testing.assert_allclose(a1[0], a2[0], rtol=1e-14)


# ---------------------------------------------------------------- TNFW
def _tnfw_rho(xi, tau):
    """Truncated NFW density in units of rho_0 at r = xi Rs."""
    return 1.0 / (xi * (1.0 + xi) ** 2) * tau * tau / (tau * tau + xi * xi)


def _cylinder_mass(X, tau):
    """Mass of the density inside the cylinder of radius X (units rho_0 Rs^3 / 4 pi):
    a shell of radius xi lies inside for xi <= X, otherwise the fraction
    1 - sqrt(1 - X^2/xi^2) of it does."""
    f = lambda xi: xi * xi * _tnfw_rho(xi, tau)
    a, _ = quad(f, 0.0, X, epsabs=0, epsrel=1e-12, limit=400)
    b, _ = quad(lambda xi: f(xi) * (1.0 - math.sqrt(1.0 - (X / xi) ** 2)), X, np.inf, epsabs=0, epsrel=1e-12,
                limit=400)
    return a + b


@pytest.mark.parametrize("tau", [0.4, 1.0, 3.0, 25.0])
@pytest.mark.parametrize("X", [0.01, 0.5, 0.97, 1.0, 1.03, 4.0, 60.0])
def test_tnfw_alpha_is_cylinder_mass(X, tau):
    # alpha(R) = M_cyl(R) / (pi R) with rho_0 = alpha_Rs / (4 Rs^2 (1 - ln 2))
    Rs, aRs = 0.2, 3e-3
    r = X * Rs
    ax, ay = O.tnfw_deflection(np.array([r]), np.array([0.0]), Rs, aRs, tau * Rs, 0.0, 0.0)
    rho0 = aRs / (4.0 * Rs * Rs * (1.0 - math.log(2.0)))
    expect = 4.0 * math.pi * rho0 * Rs ** 3 * _cylinder_mass(X, tau) / (math.pi * r)
    assert abs(ax[0] - expect) <= 1e-9 * expect
    assert ay[0] == 0.0


def test_tnfw_untruncated_limit_is_nfw():
    rng = np.random.default_rng(8)
    x, y = rng.uniform(-2, 2, (2, 300))
    Rs = np.array([0.05, 0.3, 0.9])
    aRs = np.array([1e-3, 4e-3, 2e-2])
    sx, sy = np.array([0.2, -0.5, 1.0]), np.array([0.1, 0.7, -0.4])
    a = O.tnfw_deflection(x, y, Rs, aRs, 1e7 * Rs, sx, sy)
    b = O.nfw_deflection(x, y, Rs, aRs, sx, sy)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-8, atol=1e-15)
    np.testing.assert_allclose(a[1], b[1], rtol=1e-8, atol=1e-15)


@pytest.mark.parametrize("tau", [0.5, 2.0, 15.0])
def test_tnfw_far_field_is_total_mass(tau):
    m, _ = quad(lambda xi: xi * xi * _tnfw_rho(xi, tau), 0.0, np.inf, epsabs=0, epsrel=1e-12, limit=400)
    G = O.tnfw_G(1e5, tau)
    assert abs(G - m) <= 1e-4 * m                 # the mass outside x falls as x^-2


def test_tnfw_zero_at_centre_and_linear_in_alpha_Rs():
    rng = np.random.default_rng(4)
    x, y = rng.uniform(-1, 1, (2, 50))
    x[0], y[0] = 0.3, -0.2
    a1 = O.tnfw_deflection(x, y, 0.1, 1e-3, 0.8, 0.3, -0.2)
    a3 = O.tnfw_deflection(x, y, 0.1, 3e-3, 0.8, 0.3, -0.2)
    assert a1[0][0] == 0.0 and a1[1][0] == 0.0
    np.testing.assert_allclose(a3[0], 3.0 * a1[0], rtol=1e-14)
    np.testing.assert_allclose(a3[1], 3.0 * a1[1], rtol=1e-14)


# ---------------------------------------------------------------- point mass
def test_point_mass_lens_equation_images():
    """For a source at distance b from a point lens the images lie on the
    source's radial line at (b +- sqrt(b^2 + 4 theta_E^2))/2."""
    te, b = 0.8, 0.3
    for th in ((b + math.sqrt(b * b + 4 * te * te)) / 2, (b - math.sqrt(b * b + 4 * te * te)) / 2):
        c, s = math.cos(0.6), math.sin(0.6)
        x, y = np.array([th * c + 0.1]), np.array([th * s - 0.2])
        ax, ay = O.point_mass_deflection(x, y, [te], [0.1], [-0.2])
        np.testing.assert_allclose([x[0] - ax[0] - 0.1, y[0] - ay[0] + 0.2], [b * c, b * s], atol=1e-14)


# ---------------------------------------------------------------- composition
def test_total_deflection_superposes_profiles():
    import workloads as W
    scene = W.config4_scene(n_sub=50)
    rng = np.random.default_rng(9)
    x, y = rng.uniform(-2.5, 2.5, (2, 80))
    ax, ay = O.total_deflection(x, y, scene.lens)
    s, g, n = scene.lens.sie, scene.lens.shear, scene.lens.nfw
    e1 = O.sie_deflection(x, y, s.theta_E, s.q, s.phi, s.cx, s.cy)
    e2 = O.shear_deflection(x, y, g.gamma1, g.gamma2)
    e3 = O.nfw_deflection(x, y, n.Rs, n.alpha_Rs, n.x, n.y)
    np.testing.assert_allclose(ax, e1[0] + e2[0] + e3[0], rtol=1e-14, atol=1e-15)
    bx, by = O.ray_shoot(x, y, scene.lens)
    np.testing.assert_allclose(bx, x - ax, rtol=0, atol=1e-15)
