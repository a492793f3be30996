"""Pins of the oracle's chi^2 gradient: its torch FP64 forward equals the NumPy
oracle; the autograd gradient matches FP64 central finite differences of the
NumPy oracle's log-likelihood; it vanishes at the noise-free truth; and the
amplitude derivative equals its closed form (the model is linear in amp)."""
import copy
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _small_scene(n_sub=25, s=2, lens_light=True):
    sc = W.config2_scene(n_sub=n_sub, npix=20, supersample=s, psf_size=5)
    sc.grid = W.Grid(nx=22, ny=19, pixel_scale=0.12, x0=0.03, y0=-0.02, supersample=s)
    if not lens_light:
        sc.lens_light = []
    return sc


def _data(sc, seed=0):
    m = O.simulate_image(sc)
    rng = np.random.default_rng(seed)
    d = m + 0.02 * np.abs(m).max() * rng.standard_normal(m.shape)
    return d, 1.0 / O.noise_variance(d, 0.01, 1000.0)


def _logL(sc, d, w):
    m = O.simulate_image(sc)
    return -0.5 * float(np.sum((m - d) ** 2 * w))


def _set_macro(sc, vec):
    sc = copy.deepcopy(sc)
    L = sc.lens
    L.sie = W.SIE(*vec[:5])
    L.shear = W.Shear(*vec[5:7])
    comps = list(sc.source) + list(sc.lens_light)
    new = [W.Sersic(*vec[7 + 7 * k: 14 + 7 * k]) for k in range(len(comps))]
    sc.source = new[:len(sc.source)]
    sc.lens_light = new[len(sc.source):]
    return sc


def test_torch_forward_matches_numpy_oracle():
    import torch
    from oracle import grad as G
    sc = _small_scene()
    mac = torch.tensor(O.macro_vector(sc.lens, sc.source, sc.lens_light))
    n = sc.lens.nfw
    t = lambda a: torch.tensor(np.asarray(a, np.float64))
    m = G.torch_forward(mac, t(n.x), t(n.y), t(n.alpha_Rs), t(n.Rs), sc.grid, len(sc.source),
                        len(sc.lens_light), sc.psf).numpy()
    np.testing.assert_allclose(m, O.simulate_image(sc), rtol=1e-12, atol=1e-14 * np.abs(m).max())


def _richardson(f, h):
    """Central difference at h and h/2 combined to cancel the h^2 term."""
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * d2 - d1) / 3


def test_gradient_matches_central_differences():
    sc = _small_scene()
    d, w = _data(sc)
    logL, gm, gs = O.chi2_gradient(sc, d, w)
    assert logL == pytest.approx(_logL(sc, d, w), rel=1e-12)
    vec = O.macro_vector(sc.lens, sc.source, sc.lens_light)
    names = O.macro_names(len(sc.source), len(sc.lens_light))
    for k in range(vec.size):
        def f(h, k=k):
            v = vec.copy()
            v[k] += h
            return _logL(_set_macro(sc, v), d, w)
        fd = _richardson(f, 1e-4 * max(abs(vec[k]), 0.1))
        assert abs(fd - gm[k]) <= 1e-6 * np.abs(gm).max(), (names[k], fd, gm[k])
    nfw = sc.lens.nfw
    for kk in np.argsort(-nfw.alpha_Rs)[:4]:
        for col, arr in enumerate(("x", "y", "alpha_Rs")):
            base = getattr(nfw, arr).astype(np.float64)

            def f(h, kk=kk, arr=arr, base=base):
                sc2 = copy.deepcopy(sc)
                a = base.copy()
                a[kk] += h
                setattr(sc2.lens.nfw, arr, a)
                return _logL(sc2, d, w)
            h = 1e-4 * (max(abs(base[kk]), 0.1) if arr != "alpha_Rs" else base[kk])
            fd = _richardson(f, h)
            assert abs(fd - gs[kk, col]) <= 1e-6 * np.abs(gs[:, col]).max(), (kk, arr, fd, gs[kk, col])


def test_gradient_vanishes_at_noise_free_truth():
    """Data equal to the model (up to the last bits of the two FP64 forwards):
    the gradient is ~1e-12 of its size at noisy data."""
    sc = _small_scene()
    m = O.simulate_image(sc)
    w = 1.0 / O.noise_variance(m, 0.01, 1000.0)
    logL, gm, gs = O.chi2_gradient(sc, m, w)
    d, w2 = _data(sc)
    _, gm_n, gs_n = O.chi2_gradient(sc, d, w2)
    assert abs(logL) < 1e-20
    assert np.abs(gm).max() < 1e-10 * np.abs(gm_n).max()
    assert np.abs(gs).max() < 1e-10 * np.abs(gs_n).max()


def test_amplitude_derivative_closed_form():
    """m is linear in a component's amplitude: d logL / d amp = sum w (d - m) m_k / amp."""
    sc = _small_scene(lens_light=False)
    d, w = _data(sc, seed=3)
    _, gm, _ = O.chi2_gradient(sc, d, w)
    m = O.simulate_image(sc)
    for k, c in enumerate(sc.source):
        only = copy.deepcopy(sc)
        only.source = [c]
        mk = O.simulate_image(only)
        expect = float(np.sum(w * (d - m) * mk)) / c.amp
        assert gm[7 + 7 * k] == pytest.approx(expect, rel=1e-10)


def test_shear_gradient_closed_form_without_subhalos():
    """With an SIS-free lens the shear enters alpha linearly; its gradient
    equals -sum lambda_beta . d alpha/d gamma with d alpha/d gamma1 = (x, -y),
    checked here against the NumPy model's linear response."""
    sc = _small_scene(n_sub=0)
    sc.lens.nfw = None
    d, w = _data(sc, seed=5)
    _, gm, _ = O.chi2_gradient(sc, d, w)
    h = 1e-6
    for k in (5, 6):
        vec = O.macro_vector(sc.lens, sc.source, sc.lens_light)
        vp, vm = vec.copy(), vec.copy()
        vp[k] += h
        vm[k] -= h
        fd = (_logL(_set_macro(sc, vp), d, w) - _logL(_set_macro(sc, vm), d, w)) / (2 * h)
        assert fd == pytest.approx(gm[k], rel=1e-6)


def test_torch_sie_is_zero_at_its_centre_like_the_numpy_oracle():
    # the deflection of the SIE is set to zero where psi = 0 (its centre); the
    # torch restatement must agree there, for q < 1 and in the q -> 1 series,
    # and keep finite gradients at the other points
    import torch
    from oracle import grad as G
    for q in (0.7, 1.0 - 1e-8):
        cx, cy = 0.125, -0.0625
        x = torch.tensor([cx, cx + 0.3, cx - 0.2], dtype=torch.float64)
        y = torch.tensor([cy, cy - 0.1, cy + 0.4], dtype=torch.float64)
        par = torch.tensor([1.2, q, 0.4, cx, cy], dtype=torch.float64, requires_grad=True)
        ax, ay = G._sie(torch, x, y, *par)
        ex, ey = O.sie_deflection(x.numpy(), y.numpy(), 1.2, q, 0.4, cx, cy)
        assert float(ax[0].detach()) == 0.0 and float(ay[0].detach()) == 0.0 and ex[0] == 0.0 and ey[0] == 0.0
        np.testing.assert_allclose(ax.detach().numpy(), ex, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(ay.detach().numpy(), ey, rtol=1e-12, atol=1e-15)
        (ax[1:].sum() + ay[1:].sum()).backward()
        assert bool(torch.isfinite(par.grad).all())


# ---------------------------------------------------- EPL main deflector, TNFW
def _epl_tnfw_scene(n_sub=25, s=2):
    sc = W.epl_scene(n_sub=n_sub, npix=20, supersample=s, psf_size=5)
    sc.grid = W.Grid(nx=22, ny=19, pixel_scale=0.12, x0=0.03, y0=-0.02, supersample=s)
    nfw = sc.lens.nfw
    rng = np.random.default_rng(77)
    nfw.r_trunc = (10.0 ** rng.uniform(0.5, 1.5, nfw.n) * nfw.Rs).astype(np.float32)
    return sc


def _set_macro_epl(sc, vec):
    sc = copy.deepcopy(sc)
    sc.lens.epl = W.EPL(*vec[:6])
    sc.lens.shear = W.Shear(*vec[6:8])
    comps = list(sc.source) + list(sc.lens_light)
    new = [W.Sersic(*vec[8 + 7 * k: 15 + 7 * k]) for k in range(len(comps))]
    sc.source = new[:len(sc.source)]
    sc.lens_light = new[len(sc.source):]
    return sc


def test_torch_forward_matches_numpy_oracle_epl_tnfw():
    """The torch restatement's EPL (its hypergeometric series) and truncated
    NFW against the NumPy oracle (SciPy's 2F1, the NumPy G)."""
    import torch
    from oracle import grad as G
    sc = _epl_tnfw_scene()
    assert G.main_kind(sc.lens) == "epl"
    mac = torch.tensor(O.macro_vector(sc.lens, sc.source, sc.lens_light))
    n = sc.lens.nfw
    t = lambda a: torch.tensor(np.asarray(a, np.float64))
    m = G.torch_forward(mac, t(n.x), t(n.y), t(n.alpha_Rs), t(n.Rs), sc.grid, len(sc.source),
                        len(sc.lens_light), sc.psf, "epl", t(n.r_trunc)).numpy()
    np.testing.assert_allclose(m, O.simulate_image(sc), rtol=1e-11, atol=1e-13 * np.abs(m).max())


def test_gradient_matches_central_differences_epl_tnfw():
    """Every macro parameter of an EPL + shear + Sersic scene (the slope gamma
    included) and (x, y, alpha_Rs) of the four strongest truncated subhalos
    against Richardson central differences of the NumPy oracle's log L."""
    sc = _epl_tnfw_scene()
    d, w = _data(sc, seed=2)
    logL, gm, gs = O.chi2_gradient(sc, d, w)
    assert logL == pytest.approx(_logL(sc, d, w), rel=1e-11)
    vec = O.macro_vector(sc.lens, sc.source, sc.lens_light)
    names = O.macro_names(len(sc.source), len(sc.lens_light), "epl")
    assert len(names) == vec.size == gm.size
    for k in range(vec.size):
        def f(h, k=k):
            v = vec.copy()
            v[k] += h
            return _logL(_set_macro_epl(sc, v), d, w)
        fd = _richardson(f, 1e-4 * max(abs(vec[k]), 0.1))
        assert abs(fd - gm[k]) <= 1e-6 * np.abs(gm).max(), (names[k], fd, gm[k])
    nfw = sc.lens.nfw
    for kk in np.argsort(-nfw.alpha_Rs)[:4]:
        for col, arr in enumerate(("x", "y", "alpha_Rs")):
            base = getattr(nfw, arr).astype(np.float64)

            def f(h, kk=kk, arr=arr, base=base):
                sc2 = copy.deepcopy(sc)
                a = base.copy()
                a[kk] += h
                setattr(sc2.lens.nfw, arr, a)
                return _logL(sc2, d, w)
            h = 1e-4 * (max(abs(base[kk]), 0.1) if arr != "alpha_Rs" else base[kk])
            fd = _richardson(f, h)
            assert abs(fd - gs[kk, col]) <= 1e-6 * np.abs(gs[:, col]).max(), (kk, arr, fd, gs[kk, col])


def test_epl_gradient_at_slope_two_is_the_sie_gradient():
    """At gamma = 2 the EPL is the SIE (same theta_E normalisation): its
    gradient in (theta_E, q, phi, cx, cy), the shear and the Sersic
    parameters equals the SIE scene's, and the slope derivative is finite."""
    sc = _epl_tnfw_scene(n_sub=0)
    sc.lens.nfw = None
    e = sc.lens.epl
    sc.lens.epl = W.EPL(e.theta_E, 2.0, e.q, e.phi, e.cx, e.cy)
    sie = copy.deepcopy(sc)
    sie.lens.epl = None
    sie.lens.sie = W.SIE(e.theta_E, e.q, e.phi, e.cx, e.cy)
    d, w = _data(sie, seed=4)
    _, g_epl, _ = O.chi2_gradient(sc, d, w)
    _, g_sie, _ = O.chi2_gradient(sie, d, w)
    keep = np.r_[0, 2:g_epl.size]
    np.testing.assert_allclose(g_epl[keep], g_sie, rtol=1e-8, atol=1e-10 * np.abs(g_sie).max())
    assert np.isfinite(g_epl[1])
