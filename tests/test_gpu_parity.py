"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element
by element on the same seeded FP32 inputs.

Bars: deflections e_alpha <= 1e-5, images e_I <= 1e-4 (tests/parity.py).
Sizes span several tiles and ragged tails; the full headline image (200x200
px, s = 3, 10,000 NFW, 41x41 PSF) is checked in the launch configuration the
benchmark times on all of its pixels, before and after the PSF, against the
stored oracle image; the larger images on sampled pixels the oracle computes
one by one (the floors of the error metric always come from the oracle's
values, never from the GPU's).
"""
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import DEFLECTION_TOL, IMAGE_TOL, deflection_error, image_error

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2606_01547_amd import Context
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = Context(0)
    yield c
    c.close()


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def _f32(a):
    return np.asarray(a, dtype=np.float32)


# ---------------------------------------------------------------- deflection
@pytest.mark.parametrize("draw", range(6))
def test_deflection_macro_lens(ctx, draw):
    sc = W.config1_scene(draw=draw)
    x, y = W.random_points(4099, 2.5, seed=draw)
    ax, ay = ctx.deflection(x, y, sc.lens)
    ex, ey = O.total_deflection(x, y, sc.lens)
    assert deflection_error(_np(ax), _np(ay), ex, ey) <= DEFLECTION_TOL


@pytest.mark.parametrize("q", [1.0, 1.0 - 1e-6, 0.9999, 0.995, 0.6, 0.2])
def test_deflection_sie_axis_ratios(ctx, q):
    lens = W.Lens(sie=W.SIE(1.1, q, 0.7, 0.03, -0.02))
    x, y = W.random_points(3000, 2.0, seed=11)
    ax, ay = ctx.deflection(x, y, lens)
    ex, ey = O.total_deflection(x, y, lens)
    assert deflection_error(_np(ax), _np(ay), ex, ey) <= DEFLECTION_TOL


# the EPL is evaluated in FP64 on the device: only the FP32 rounding of the
# output separates it from the oracle
EPL_TOL = 1e-6


@pytest.mark.parametrize("gamma,q", [(1.2, 0.3), (1.5, 0.6), (2.0, 0.8), (2.5, 0.95), (2.8, 1.0), (1.9, 0.05),
                                     (2.05, 1.0 - 1e-7)])
def test_deflection_epl_slopes_and_axis_ratios(ctx, gamma, q):
    cx, cy = 0.03125, -0.015625          # exact in FP32, so one point is the centre itself
    lens = W.Lens(epl=W.EPL(1.05, gamma, q, 0.7, cx, cy))
    x, y = W.random_points(3001, 2.0, seed=13)
    x[:3] = [cx, 0.5, -1.0]
    y[:3] = [cy, cy, cy]
    ax, ay = ctx.deflection(x, y, lens)
    ex, ey = O.total_deflection(x, y, lens)
    ax, ay = _np(ax), _np(ay)
    assert ax[0] == 0.0 and ay[0] == 0.0
    assert deflection_error(ax, ay, ex, ey) <= EPL_TOL


def test_epl_gamma_two_matches_the_sie_kernel(ctx):
    x, y = W.random_points(4096, 2.0, seed=17)
    for q in (0.35, 0.8, 1.0):
        a = ctx.deflection(x, y, W.Lens(epl=W.EPL(1.2, 2.0, q, 0.4, 0.1, -0.05)))
        b = ctx.deflection(x, y, W.Lens(sie=W.SIE(1.2, q, 0.4, 0.1, -0.05)))
        assert deflection_error(_np(a[0]), _np(a[1]), _np(b[0]), _np(b[1])) <= EPL_TOL


def test_epl_with_sie_shear_and_subhalos_superposes(ctx):
    sc = W.epl_scene(n_sub=300)
    lens = sc.lens
    lens.sie = W.SIE(0.3, 0.7, 1.1, -0.2, 0.1)
    x, y = W.random_points(2049, 2.5, seed=19)
    ax, ay = ctx.deflection(x, y, lens)
    ex, ey = O.total_deflection(x, y, lens)
    assert deflection_error(_np(ax), _np(ay), ex, ey) <= DEFLECTION_TOL


def test_epl_rejects_bad_parameters(ctx):
    from paper_2606_01547_amd import JtError
    x, y = W.random_points(16, 1.0, seed=1)
    for e in (W.EPL(1.0, 1.0, 0.8, 0, 0, 0), W.EPL(1.0, 3.0, 0.8, 0, 0, 0), W.EPL(-1.0, 2.0, 0.8, 0, 0, 0),
              W.EPL(1.0, 2.0, 0.0, 0, 0, 0), W.EPL(1.0, 2.0, 0.01, 0, 0, 0), W.EPL(1.0, float("nan"), 0.8, 0, 0, 0)):
        with pytest.raises(JtError):
            ctx.deflection(x, y, W.Lens(epl=e))


def test_deflection_point_masses_and_shear(ctx):
    pm = W.PointMasses(x=np.array([0.3, -0.5, 1.1]), y=np.array([0.1, 0.4, -0.9]),
                       theta_E=np.array([0.4, 0.2, 0.1]))
    lens = W.Lens(shear=W.Shear(0.02, -0.03), point_masses=pm)
    x, y = W.random_points(2000, 2.0, seed=3)
    ax, ay = ctx.deflection(x, y, lens)
    ex, ey = O.total_deflection(x, y, lens)
    assert deflection_error(_np(ax), _np(ay), ex, ey) <= DEFLECTION_TOL


def _near_points(nfw, rng, count):
    """Points at r = X Rs around random subhalos, X spanning every branch of the
    NFW term (centre, small x, x -> 1 from both sides, far)."""
    idx = rng.integers(0, nfw.n, count)
    X = rng.choice([0.0, 1e-3, 0.05, 0.3, 0.5, 0.7, 0.9, 0.95, 0.999, 1.0, 1.001, 1.05, 1.5, 3.0], count)
    ang = rng.uniform(0, 2 * np.pi, count)
    x = nfw.x[idx].astype(np.float64) + X * nfw.Rs[idx] * np.cos(ang)
    y = nfw.y[idx].astype(np.float64) + X * nfw.Rs[idx] * np.sin(ang)
    return _f32(x), _f32(y)


def test_deflection_headline_subhalos(ctx):
    sc = W.config2_scene()
    rng = np.random.default_rng(5)
    x1, y1 = W.random_points(1500, 5.0, seed=21)
    x2, y2 = _near_points(sc.lens.nfw, rng, 700)
    x, y = np.concatenate([x1, x2]), np.concatenate([y1, y2])
    ax, ay = ctx.deflection(x, y, sc.lens)
    ex, ey = O.total_deflection(x, y, sc.lens)
    assert deflection_error(_np(ax), _np(ay), ex, ey) <= DEFLECTION_TOL


@pytest.mark.parametrize("nsub", [0, 1, 2, 3, 5, 63, 64, 65, 129])
@pytest.mark.parametrize("npts", [1, 255, 257])
def test_deflection_ragged_counts(ctx, nsub, npts):
    sc = W.config4_scene(n_sub=max(nsub, 1))
    nfw = sc.lens.nfw
    if nsub == 0:
        nfw = W.NFWTable(nfw.x[:0], nfw.y[:0], nfw.Rs[:0], nfw.alpha_Rs[:0])
    lens = W.Lens(sie=sc.lens.sie, shear=sc.lens.shear, nfw=nfw)
    x, y = W.random_points(npts, 3.0, seed=nsub * 1000 + npts)
    ax, ay = ctx.deflection(x, y, lens)
    ex, ey = O.total_deflection(x, y, lens)
    assert deflection_error(_np(ax), _np(ay), ex, ey) <= DEFLECTION_TOL


def test_subhalos_alone(ctx):
    """NFW sum without the macro lens: the subhalo term itself meets the bar."""
    sc = W.config2_scene(n_sub=2000)
    lens = W.Lens(nfw=sc.lens.nfw)
    rng = np.random.default_rng(8)
    x1, y1 = W.random_points(1000, 3.5, seed=4)
    x2, y2 = _near_points(sc.lens.nfw, rng, 500)
    x, y = np.concatenate([x1, x2]), np.concatenate([y1, y2])
    ax, ay = ctx.deflection(x, y, lens)
    ex, ey = O.total_deflection(x, y, lens)
    assert deflection_error(_np(ax), _np(ay), ex, ey) <= DEFLECTION_TOL


def test_single_nfw_every_branch(ctx):
    """One subhalo, points at r = X Rs across the near-field forms (series
    near x = 1, log1p form below), the far-field polynomial and the centre:
    per-point relative error of the deflection."""
    Rs, aRs, cx, cy = 0.1, 2e-3, 0.3, -0.2
    X = np.array([1e-3, 0.01, 0.05, 0.1, 0.2, 0.3, 0.49, 0.5, 0.51, 0.7, 0.85, 0.89, 0.9, 0.91, 0.95,
                  0.99, 0.999, 1.0, 1.001, 1.01, 1.1, 1.5, 2.0, 5.0, 50.0, 500.0])
    ang = np.linspace(0.1, 6.0, X.size)
    x = _f32(cx + X * Rs * np.cos(ang))
    y = _f32(cy + X * Rs * np.sin(ang))
    nfw = W.NFWTable(_f32([cx]), _f32([cy]), _f32([Rs]), _f32([aRs]))
    lens = W.Lens(nfw=nfw)
    ax, ay = ctx.deflection(x, y, lens)
    ex, ey = O.total_deflection(x, y, lens)
    rel = np.hypot(_np(ax) - ex, _np(ay) - ey) / np.hypot(ex, ey)
    assert rel.max() <= 5e-6, dict(zip(X.tolist(), rel.tolist()))
    a0 = ctx.deflection(_f32([cx]), _f32([cy]), lens)
    assert _np(a0[0])[0] == 0.0 and _np(a0[1])[0] == 0.0


def test_deflection_independent_of_launch_split(ctx):
    """The summation order is fixed: a few points (launched with the subhalo
    quarters spread over 4 waves) and the same points inside a large batch
    (one wave per point) give bitwise the same deflection."""
    sc = W.config2_scene()
    x, y = W.random_points(100, 4.0, seed=12)
    bx, by = W.random_points(2_000_000, 4.0, seed=13)
    small = ctx.deflection(x, y, sc.lens)
    big = ctx.deflection(np.concatenate([x, bx]), np.concatenate([y, by]), sc.lens)
    np.testing.assert_array_equal(_np(small[0]), _np(big[0])[:100])
    np.testing.assert_array_equal(_np(small[1]), _np(big[1])[:100])


def test_truncated_deflection_independent_of_launch_split(ctx):
    """The truncated profile's records pass through a per-wave LDS stage whose
    length follows the launch's wave split (8 records with two wave-groups, 32
    otherwise): the same 100 points alone (split 8) and at the head of batches
    launched with splits 4, 2 and 1 give bitwise the same deflection."""
    sc = W.tnfw_scene(n_sub=2000)
    x, y = W.random_points(100, 4.0, seed=14)
    small = ctx.deflection(x, y, sc.lens)
    for n, seed in ((600_000, 15), (1_200_000, 16), (2_200_000, 17)):
        bx, by = W.random_points(n, 4.0, seed=seed)
        big = ctx.deflection(np.concatenate([x, bx]), np.concatenate([y, by]), sc.lens)
        np.testing.assert_array_equal(_np(small[0]), _np(big[0])[:100])
        np.testing.assert_array_equal(_np(small[1]), _np(big[1])[:100])


def test_resident_table_matches_device_soa_bitwise(ctx):
    sc = W.config2_scene(n_sub=777)
    x, y = W.random_points(5000, 4.0, seed=1)
    a1 = ctx.deflection(x, y, sc.lens)
    h = ctx.upload_subhalos(sc.lens.nfw)
    lens_h = W.Lens(sie=sc.lens.sie, shear=sc.lens.shear)
    lens_h.subhalo_handle = h
    a2 = ctx.deflection(x, y, lens_h)
    np.testing.assert_array_equal(_np(a1[0]), _np(a2[0]))
    np.testing.assert_array_equal(_np(a1[1]), _np(a2[1]))
    ctx.release(h)


# ---------------------------------------------------------------- TNFW subhalos
@pytest.mark.parametrize("tau", [0.4, 1.0, 3.0, 25.0, 300.0])
def test_single_tnfw_every_branch(ctx, tau):
    """One truncated subhalo, points at r = X Rs across the log1p form, the
    series near x = 1, the arctangent form and the far field: per-point
    relative error of the deflection."""
    Rs, aRs, cx, cy = 0.1, 2e-3, 0.3, -0.2
    X = np.array([1e-3, 0.01, 0.05, 0.2, 0.5, 0.85, 0.89, 0.9, 0.95, 0.999, 1.0, 1.001, 1.05, 1.09, 1.1, 1.2,
                  1.5, 2.0, 5.0, 50.0, 500.0, 3000.0])
    ang = np.linspace(0.1, 6.0, X.size)
    x = _f32(cx + X * Rs * np.cos(ang))
    y = _f32(cy + X * Rs * np.sin(ang))
    nfw = W.NFWTable(_f32([cx]), _f32([cy]), _f32([Rs]), _f32([aRs]), r_trunc=_f32([tau * Rs]))
    lens = W.Lens(nfw=nfw)
    ax, ay = ctx.deflection(x, y, lens)
    ex, ey = O.total_deflection(x, y, lens)
    rel = np.hypot(_np(ax) - ex, _np(ay) - ey) / np.hypot(ex, ey)
    assert rel.max() <= 1e-5, dict(zip(X.tolist(), rel.tolist()))
    a0 = ctx.deflection(_f32([cx]), _f32([cy]), lens)
    assert _np(a0[0])[0] == 0.0 and _np(a0[1])[0] == 0.0


@pytest.mark.parametrize("tau", [0.4, 2.0, 7.0, 40.0, 300.0, 1e4])
def test_single_tnfw_far_field_boundary(ctx, tau):
    """Points just inside and outside x_f = max(0.75 tau, 1.5), where the pair
    switches between the general form and the far-field polynomial, and far
    beyond it: per-point relative error of the deflection."""
    Rs, aRs, cx, cy = 0.1, 2e-3, 0.3, -0.2
    xf = max(0.75 * tau, 1.5)
    X = xf * np.array([0.95, 0.99, 0.999, 1.0005, 1.001, 1.01, 1.1, 1.5, 3.0, 10.0, 100.0, 1000.0])
    ang = np.linspace(0.2, 6.1, X.size)
    x = _f32(cx + X * Rs * np.cos(ang))
    y = _f32(cy + X * Rs * np.sin(ang))
    lens = W.Lens(nfw=W.NFWTable(_f32([cx]), _f32([cy]), _f32([Rs]), _f32([aRs]), r_trunc=_f32([tau * Rs])))
    ax, ay = ctx.deflection(x, y, lens)
    ex, ey = O.total_deflection(x, y, lens)
    rel = np.hypot(_np(ax) - ex, _np(ay) - ey) / np.hypot(ex, ey)
    assert rel.max() <= 1e-5, dict(zip((X / xf).tolist(), rel.tolist()))


def test_deflection_truncated_subhalos_full_lens(ctx):
    sc = W.tnfw_scene()
    rng = np.random.default_rng(6)
    x1, y1 = W.random_points(1500, 5.0, seed=22)
    x2, y2 = _near_points(sc.lens.nfw, rng, 700)
    x, y = np.concatenate([x1, x2]), np.concatenate([y1, y2])
    ax, ay = ctx.deflection(x, y, sc.lens)
    ex, ey = O.total_deflection(x, y, sc.lens)
    assert deflection_error(_np(ax), _np(ay), ex, ey) <= DEFLECTION_TOL
    alone = W.Lens(nfw=sc.lens.nfw)
    ax, ay = ctx.deflection(x, y, alone)
    ex, ey = O.total_deflection(x, y, alone)
    assert deflection_error(_np(ax), _np(ay), ex, ey) <= DEFLECTION_TOL


@pytest.mark.parametrize("nsub", [1, 3, 5, 64, 65])
def test_truncated_subhalos_ragged_counts(ctx, nsub):
    sc = W.tnfw_scene(n_sub=nsub, npix=20)
    x, y = W.random_points(257, 3.0, seed=nsub)
    ax, ay = ctx.deflection(x, y, sc.lens)
    ex, ey = O.total_deflection(x, y, sc.lens)
    assert deflection_error(_np(ax), _np(ay), ex, ey) <= DEFLECTION_TOL


def test_weakly_truncated_subhalos_match_the_nfw_kernel(ctx):
    # tau = 1e6: the truncation changes these deflections by ~4e-9 (1e4 would
    # already give ~2e-5), so the two kernels must agree to the bar
    sc = W.config2_scene(n_sub=1000)
    nfw = sc.lens.nfw
    t = W.NFWTable(nfw.x, nfw.y, nfw.Rs, nfw.alpha_Rs, r_trunc=_f32(1e6 * nfw.Rs))
    x, y = W.random_points(3000, 4.0, seed=3)
    a = ctx.deflection(x, y, W.Lens(nfw=t))
    b = ctx.deflection(x, y, W.Lens(nfw=nfw))
    assert deflection_error(_np(a[0]), _np(a[1]), _np(b[0]), _np(b[1])) <= DEFLECTION_TOL


def test_truncated_resident_table_matches_device_soa_bitwise(ctx):
    sc = W.tnfw_scene(n_sub=777)
    x, y = W.random_points(5000, 4.0, seed=1)
    a1 = ctx.ray_shoot(x, y, sc.lens)
    h = ctx.upload_subhalos(sc.lens.nfw)
    lens_h = W.Lens(sie=sc.lens.sie, shear=sc.lens.shear)
    lens_h.subhalo_handle = h
    a2 = ctx.ray_shoot(x, y, lens_h)
    np.testing.assert_array_equal(_np(a1[0]), _np(a2[0]))
    np.testing.assert_array_equal(_np(a1[1]), _np(a2[1]))
    ctx.release(h)


def test_truncated_upload_rejects_bad_radii(ctx):
    from paper_2606_01547_amd import JtError
    sc = W.tnfw_scene(n_sub=10, npix=20)
    for bad in (0.0, -1.0, float("nan")):
        nfw = sc.lens.nfw
        rt = nfw.r_trunc.copy()
        rt[3] = bad
        with pytest.raises(JtError):
            ctx.upload_subhalos(W.NFWTable(nfw.x, nfw.y, nfw.Rs, nfw.alpha_Rs, r_trunc=rt))


def test_ray_shoot_is_theta_minus_alpha(ctx):
    sc = W.config2_scene(n_sub=500)
    x, y = W.random_points(3333, 4.0, seed=2)
    bx, by = ctx.ray_shoot(x, y, sc.lens)
    ax, ay = ctx.deflection(x, y, sc.lens)
    # both round one FP64 alpha: beta = fl(theta - alpha), alpha_out = fl(alpha)
    for b, t, a in ((_np(bx), x, _np(ax)), (_np(by), y, _np(ay))):
        bound = 0.5 * np.spacing(np.abs(b).astype(np.float32)) + 0.5 * np.spacing(np.abs(a).astype(np.float32))
        assert np.all(np.abs(b - (t.astype(np.float64) - a)) <= bound)
    ex, ey = O.ray_shoot(x, y, sc.lens)
    gx, gy = _np(bx), _np(by)
    # beta parity expressed on alpha = theta - beta (FP32 rounding of beta included)
    assert deflection_error(x - gx, y - gy, x - ex, y - ey) <= DEFLECTION_TOL


def test_empty_point_set(ctx):
    sc = W.config1_scene()
    e = np.zeros(0, np.float32)
    ax, ay = ctx.deflection(e, e, sc.lens)
    assert ax.numel() == 0


# ---------------------------------------------------------------- surface brightness
@pytest.mark.parametrize("bn_exact", [False, True])
def test_source_sb_stage_isolated(ctx, bn_exact):
    sc = W.config2_scene(n_sub=10)
    x, y = W.random_points(10001, 3.0, seed=7)
    bx, by = W.random_points(10001, 1.0, seed=8)
    sb = ctx.source_sb(x, y, bx, by, sc.source, sc.lens_light, bn_exact=bn_exact)
    ref = O.surface_brightness(x, y, bx, by, sc.source, sc.lens_light, bn_exact)
    assert image_error(_np(sb), ref) <= 2e-5


def test_source_sb_at_gpu_traced_points(ctx):
    sc = W.config2_scene(n_sub=3000)
    x, y = W.random_points(4000, 3.0, seed=9)
    bx, by = ctx.ray_shoot(x, y, sc.lens)
    sb = ctx.source_sb(x, y, bx, by, sc.source, sc.lens_light)
    ref = O.surface_brightness(x, y, _np(bx), _np(by), sc.source, sc.lens_light)
    assert image_error(_np(sb), ref) <= 2e-5


@pytest.mark.parametrize("n", [1, 3, 4, 5, 257, 1030])
def test_source_sb_ragged_and_unaligned_points(ctx, n):
    # 16-byte aligned arrays take four points per thread (and one per thread
    # for the last n mod 4); views starting one element in take one per
    # thread: the two give the same bits, and both match the oracle
    sc = W.config2_scene(n_sub=10)
    x, y = W.random_points(n + 1, 3.0, seed=11)
    bx, by = W.random_points(n + 1, 1.0, seed=12)
    dev = [torch.from_numpy(np.asarray(a, np.float32)).cuda() for a in (x, y, bx, by)]
    vec = ctx.source_sb(*[t[:n] for t in dev], sc.source, sc.lens_light)
    one = ctx.source_sb(*[t[1:] for t in dev], sc.source, sc.lens_light)
    ref = O.surface_brightness(x[:n], y[:n], bx[:n], by[:n], sc.source, sc.lens_light, False)
    assert image_error(_np(vec), ref) <= 2e-5
    ref1 = O.surface_brightness(x[1:], y[1:], bx[1:], by[1:], sc.source, sc.lens_light, False)
    assert image_error(_np(one), ref1) <= 2e-5
    if n > 1:
        np.testing.assert_array_equal(_np(vec)[1:], _np(
            ctx.source_sb(*[t[1:n] for t in dev], sc.source, sc.lens_light)))


def test_source_sb_reads_no_coordinates_of_an_empty_list(ctx):
    # through the C ABI: the traced coordinates may be NULL without sources,
    # and all four when both lists are empty
    from ctypes import byref, c_void_p
    from paper_2606_01547_amd._native import _stream_handle
    sc = W.config2_scene(n_sub=10)
    x, y = W.random_points(1001, 3.0, seed=13)
    xt = torch.from_numpy(np.asarray(x, np.float32)).cuda()
    yt = torch.from_numpy(np.asarray(y, np.float32)).cuda()
    keep = []
    none, ll = ctx._light([], False, keep), ctx._light(sc.lens_light, False, keep)
    sb = torch.full((1001,), 7.0, dtype=torch.float32, device="cuda")
    lib, st = ctx._lib, _stream_handle(None)
    assert lib.jt_source_sb(ctx._ptr, 1001, c_void_p(xt.data_ptr()), c_void_p(yt.data_ptr()), None, None,
                            byref(none), byref(ll), c_void_p(sb.data_ptr()), st) == 0
    ref = O.surface_brightness(x, y, x, y, [], sc.lens_light, False)
    assert image_error(_np(sb), ref) <= 2e-5
    assert lib.jt_source_sb(ctx._ptr, 1001, None, None, None, None, byref(none), byref(none),
                            c_void_p(sb.data_ptr()), st) == 0
    assert np.all(_np(sb) == 0.0)


# ---------------------------------------------------------------- convolution
@pytest.mark.parametrize("shape,k", [((53, 77), 1), ((53, 77), 3), ((53, 77), 11), ((200, 200), 41),
                                     ((64, 64), 101), ((300, 33), 129), ((9, 300), 255), ((1, 1), 5)])
def test_convolve_direct(ctx, shape, k):
    rng = np.random.default_rng(k)
    img = rng.uniform(0, 1, shape).astype(np.float32)
    psf = rng.uniform(0, 1, (k, k))
    psf[0, :] *= 3.0          # asymmetric: a correlation would fail
    psf = (psf / psf.sum()).astype(np.float32)
    out = ctx.convolve(img, psf, method=1)
    ref = O.convolve_same(img, psf)
    assert image_error(_np(out), ref) <= (2e-5 if k <= 41 else IMAGE_TOL)


@pytest.mark.parametrize("shape,k", [((53, 77), 1), ((53, 77), 11), ((200, 200), 41), ((64, 64), 101),
                                     ((300, 33), 129), ((9, 300), 255), ((1, 1), 5), ((3, 1998), 101)])
def test_convolve_fft(ctx, shape, k):
    """FP64 transforms: only the FP32 rounding of the output remains."""
    rng = np.random.default_rng(k + 7)
    img = rng.uniform(0, 1, shape).astype(np.float32)
    psf = rng.uniform(0, 1, (k, k))
    psf[:, -1] *= 4.0         # asymmetric along x
    psf[0, :] *= 3.0          # and along y
    psf = (psf / psf.sum()).astype(np.float32)
    out = ctx.convolve(img, psf, method=2)
    assert image_error(_np(out), O.convolve_same(img, psf)) <= 1e-6


def test_convolve_large_image_both_paths(ctx):
    """1000 x 1000 px with a 101 x 101 PSF (the largest workload): both paths
    on 4000 sampled pixels (every border and corner included) against the
    oracle one pixel at a time, and against each other on every pixel; method
    0 returns one of the two bit for bit."""
    rng = np.random.default_rng(5)
    n, k = 1000, 101
    img = rng.uniform(0, 1, (n, n)).astype(np.float32)
    psf = W.gaussian_psf(k, 12.0)
    psf[k // 2 + 3, :] += 1e-3     # a ridge off the centre row breaks the symmetry
    psf = (psf / psf.sum()).astype(np.float32)
    rows = np.concatenate([rng.integers(0, n, 3600), [0, 0, n - 1, n - 1], rng.integers(0, n, 396)])
    cols = np.concatenate([rng.integers(0, n, 3600), [0, n - 1, 0, n - 1], np.zeros(198, int),
                           np.full(198, n - 1)])
    ref = O.convolve_at(img, psf, rows, cols)
    direct = _np(ctx.convolve(img, psf, method=1))
    fft = _np(ctx.convolve(img, psf, method=2))
    for got in (direct, fft):
        assert image_error(got[rows, cols], ref) <= 2e-5
    assert image_error(direct, fft) <= 2e-5
    auto = _np(ctx.convolve(img, psf, method=0))
    assert np.array_equal(auto, direct) or np.array_equal(auto, fft)


def _conv_shape_kind(nx, ny):
    """The direct path's launch shape for an nx x ny image: 0 = four 16-column
    groups per block (>= 512 such blocks), 1 = two groups with two waves each
    (>= 512 such blocks), 2 = one group split over eight waves."""
    ty = (ny + 15) // 16
    if (nx + 63) // 64 * ty >= 512:
        return 0
    return 1 if (nx + 31) // 32 * ty >= 512 else 2


@pytest.mark.parametrize("nx,ny,k,kind", [(1024, 512, 21, 0), (1024, 496, 21, 1), (512, 512, 41, 1),
                                          (512, 496, 41, 2), (1000, 517, 255, 0), (1003, 301, 129, 1),
                                          (1000, 517, 3, 0)])
def test_convolve_direct_every_launch_shape(ctx, nx, ny, k, kind):
    """Each of the direct path's three launch shapes, on both sides of the
    tile counts that select them, with ragged edges, and with kernels whose
    window needs several LDS-staged row chunks (k = 255 on the four-group
    shape stages only 8 input rows at a time): 2000 sampled pixels (corners
    and every border included) against the oracle one pixel at a time."""
    assert _conv_shape_kind(nx, ny) == kind
    rng = np.random.default_rng(nx + 7 * ny + k)
    img = rng.uniform(-0.5, 1.0, (ny, nx)).astype(np.float32)
    psf = rng.uniform(0, 1, (k, k))
    psf[0, :] *= 3.0
    psf[:, -1] *= 2.0
    psf = (psf / psf.sum()).astype(np.float32)
    m = 1600
    rows = np.concatenate([rng.integers(0, ny, m), [0, 0, ny - 1, ny - 1], rng.integers(0, ny, 98),
                           np.zeros(98, int), np.full(100, ny - 1)])
    cols = np.concatenate([rng.integers(0, nx, m), [0, nx - 1, 0, nx - 1], np.zeros(98, int),
                           rng.integers(0, nx, 98), rng.integers(0, nx, 100)])
    got = _np(ctx.convolve(img, psf, method=1))
    assert image_error(got[rows, cols], O.convolve_at(img, psf, rows, cols)) <= (2e-5 if k <= 41 else IMAGE_TOL)


def test_convolve_fft_size_limit(ctx):
    from paper_2606_01547_amd import JtError
    img = np.ones((1, 2000), np.float32)
    psf = np.full((101, 101), 1.0 / 101**2, np.float32)
    with pytest.raises(JtError):
        ctx.convolve(img, psf, method=2)      # padded row of 2050 > 2048
    out = _np(ctx.convolve(img, psf, method=0))   # auto falls back to the direct path
    assert image_error(out, O.convolve_same(img, psf)) <= 2e-5


def test_convolve_delta_is_identity(ctx):
    img = np.random.default_rng(0).standard_normal((70, 90)).astype(np.float32)
    psf = np.zeros((9, 9), np.float32)
    psf[4, 4] = 1.0
    out = ctx.convolve(img, psf)
    np.testing.assert_array_equal(_np(out).astype(np.float32), img)


# ---------------------------------------------------------------- fused simulation
@pytest.mark.parametrize("draw", range(4))
def test_simulate_plain_case(ctx, draw):
    sc = W.config1_scene(draw=draw)
    got = _np(ctx.simulate_scene(sc))
    assert image_error(got, O.simulate_image(sc)) <= IMAGE_TOL


def test_simulate_differentiation_case_forward(ctx):
    sc = W.config4_scene()
    got = _np(ctx.simulate_scene(sc))
    assert image_error(got, O.simulate_image(sc)) <= IMAGE_TOL


def test_simulate_headline_physics_reduced_grid(ctx):
    sc = W.config2_scene(npix=44, n_sub=4000)
    sc.grid = W.Grid(nx=44, ny=37, pixel_scale=0.05, x0=0.11, y0=-0.07, supersample=3)
    got = _np(ctx.simulate_scene(sc))
    assert image_error(got, O.simulate_image(sc)) <= IMAGE_TOL
    un = _np(ctx.simulate_scene(sc, psf=False))
    assert image_error(un, O.simulate_unconvolved(sc)) <= IMAGE_TOL


def test_simulate_epl_scene_reduced_grid(ctx):
    sc = W.epl_scene(npix=40, n_sub=3000)
    sc.grid = W.Grid(nx=40, ny=33, pixel_scale=0.05, x0=-0.06, y0=0.09, supersample=3)
    got = _np(ctx.simulate_scene(sc))
    assert image_error(got, O.simulate_image(sc)) <= IMAGE_TOL


def test_simulate_truncated_subhalo_scene_reduced_grid(ctx):
    sc = W.tnfw_scene(npix=40, n_sub=3000)
    sc.grid = W.Grid(nx=40, ny=35, pixel_scale=0.05, x0=0.07, y0=-0.04, supersample=3)
    got = _np(ctx.simulate_scene(sc))
    assert image_error(got, O.simulate_image(sc)) <= IMAGE_TOL


def _oracle_pixels(sc, rows, cols):
    g = sc.grid
    tx, ty = O.subpixel_coords(g.nx, g.ny, g.pixel_scale, g.x0, g.y0, g.supersample)
    tx, ty = tx[rows, cols], ty[rows, cols]
    bx, by = O.ray_shoot(tx, ty, sc.lens)
    sb = O.surface_brightness(tx, ty, bx, by, sc.source, sc.lens_light, sc.bn_exact)
    return g.pixel_scale ** 2 * sb.mean(axis=(-2, -1))


def test_simulate_headline_whole_image(ctx):
    """200x200 px, s = 3, 10,000 NFW, 41x41 PSF, in the bench's launch: every
    one of the 40,000 pixels against the stored FP64 oracle image
    (tests/golden/c2_headline.npz, written by tests/golden/make_c2.py from the
    oracle alone), before and after the PSF."""
    z = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_headline.npz"))
    ref_un, ref_full = z["unconvolved"], z["convolved"]
    sc = W.config2_scene()
    un = _np(ctx.simulate_scene(sc, psf=False))
    assert image_error(un, ref_un) <= IMAGE_TOL
    full = _np(ctx.simulate_scene(sc))
    assert image_error(full, ref_full) <= IMAGE_TOL
    # the PSF step of the fused call equals jt_convolve of the unconvolved image
    np.testing.assert_array_equal(full, _np(ctx.convolve(un.astype(np.float32), sc.psf)))
    assert image_error(full, O.convolve_same(un, sc.psf)) <= 2e-5


@pytest.mark.parametrize("make", [W.epl_scene, W.tnfw_scene], ids=["epl", "tnfw"])
def test_profile_scenes_full_size_sampled(ctx, make):
    """The bench's EPL and truncated-subhalo images (200x200 px, s = 3, 10,000
    subhalos, 41x41 PSF) in the bench's launch, on sampled pixels."""
    sc = make()
    un = _np(ctx.simulate_scene(sc, psf=False))
    rng = np.random.default_rng(3)
    rows = rng.integers(0, 200, 160)
    cols = rng.integers(0, 200, 160)
    flat = np.argsort(un.reshape(-1))[-30:]
    rows = np.concatenate([rows, flat // 200])
    cols = np.concatenate([cols, flat % 200])
    ref = _oracle_pixels(sc, rows, cols)
    floor = 1e-3 * np.abs(ref).max()
    err = np.max(np.abs(un[rows, cols] - ref) / np.maximum(np.abs(ref), floor))
    assert err <= IMAGE_TOL


def _oracle_pixels_direct(sc, rows, cols):
    """Sampled pixels of a large grid without forming its whole sub-pixel
    array: pixel (i, j) is the 1 x 1 grid centred on that pixel."""
    g = sc.grid
    out = np.empty(len(rows))
    for t, (i, j) in enumerate(zip(rows, cols)):
        x0 = g.x0 + (j - (g.nx - 1) / 2.0) * g.pixel_scale
        y0 = g.y0 + (i - (g.ny - 1) / 2.0) * g.pixel_scale
        tx, ty = O.subpixel_coords(1, 1, g.pixel_scale, x0, y0, g.supersample)
        bx, by = O.ray_shoot(tx, ty, sc.lens)
        sb = O.surface_brightness(tx, ty, bx, by, sc.source, sc.lens_light, sc.bn_exact)
        out[t] = g.pixel_scale ** 2 * sb.mean()
    return out


def test_simulate_large_image_sampled(ctx):
    """1000x1000 px, s = 5, 50,000 NFW, four Sersic components, 101x101 PSF
    (the largest workload): the unconvolved image on sampled pixels against the
    oracle pixel by pixel; the convolution stage on sampled outputs."""
    sc = W.config5_scene()
    n = sc.grid.nx
    un = _np(ctx.simulate_scene(sc, psf=False))
    rng = np.random.default_rng(1)
    flat = np.argsort(un.reshape(-1))[-40:]
    rows = np.concatenate([rng.integers(0, n, 56), [0, n - 1], flat // n])
    cols = np.concatenate([rng.integers(0, n, 56), [n - 1, 0], flat % n])
    ref = _oracle_pixels_direct(sc, rows, cols)
    floor = 1e-3 * np.abs(ref).max()
    assert np.max(np.abs(un[rows, cols] - ref) / np.maximum(np.abs(ref), floor)) <= IMAGE_TOL
    full = _np(ctx.simulate_scene(sc))
    np.testing.assert_array_equal(full, _np(ctx.convolve(un.astype(np.float32), sc.psf)))
    top = np.argsort(full.reshape(-1))[-20:]
    r2 = np.concatenate([rng.integers(0, n, 300), top // n])
    c2 = np.concatenate([rng.integers(0, n, 300), top % n])
    conv_ref = O.convolve_at(un.astype(np.float32), sc.psf, r2, c2)
    fl2 = 1e-3 * np.abs(conv_ref).max()
    assert np.max(np.abs(full[r2, c2] - conv_ref) / np.maximum(np.abs(conv_ref), fl2)) <= 2e-5


def test_simulate_is_deterministic(ctx):
    sc = W.config2_scene(npix=64, n_sub=3000)
    a = _np(ctx.simulate_scene(sc))
    b = _np(ctx.simulate_scene(sc))
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("nx,ny,s", [(1, 1, 1), (1, 37, 3), (23, 5, 5), (7, 6, 16), (16, 16, 2)])
def test_simulate_grid_edge_cases(ctx, nx, ny, s):
    sc = W.config2_scene(n_sub=200)
    sc.grid = W.Grid(nx=nx, ny=ny, pixel_scale=0.07, x0=0.2, y0=0.1, supersample=s)
    got = _np(ctx.simulate_scene(sc, psf=False))
    assert image_error(got, O.simulate_unconvolved(sc)) <= IMAGE_TOL


def test_simulate_without_light_or_lens(ctx):
    sc = W.config1_scene()
    empty = W.Scene(grid=sc.grid, lens=W.Lens(), source=[], lens_light=[], psf=None)
    assert np.all(_np(ctx.simulate_scene(empty)) == 0.0)
    ll = W.Sersic(amp=2.0, R_sersic=0.6, n_sersic=3.0, q=0.8, phi=0.3, cx=0.0, cy=0.0)
    only = W.Scene(grid=sc.grid, lens=W.Lens(), source=[], lens_light=[ll], psf=sc.psf)
    assert image_error(_np(ctx.simulate_scene(only)), O.simulate_image(only)) <= IMAGE_TOL


# ---------------------------------------------------------------- argument errors
def test_overlapping_outputs_are_rejected_and_in_place_sb_is_exact(ctx):
    from paper_2606_01547_amd import JtError
    from paper_2606_01547_amd._native import JT_EINVAL
    sc = W.config2_scene(n_sub=10)
    buf = torch.from_numpy(np.concatenate(W.random_points(1500, 2.0, seed=21))).cuda()   # 3000 floats
    x, y = buf[:1000], buf[1000:2000]
    for out in ((buf[500:1500], buf[2000:3000]), (buf[2000:3000], buf[1999:2999]), (buf[1000:2000], buf[2000:3000])):
        with pytest.raises(JtError) as e:
            ctx.ray_shoot(x, y, sc.lens, out=out)
        assert e.value.status == JT_EINVAL
    img = torch.zeros(2 * 64 * 64, device="cuda")
    psf = torch.full((5, 5), 1.0 / 25, device="cuda")
    with pytest.raises(JtError) as e:
        ctx.convolve(img[:4096].view(64, 64), psf, out=img[100:4196].view(64, 64))
    assert e.value.status == JT_EINVAL
    bx = torch.empty(1001, device="cuda")
    bx[:1000] = buf[2000:3000]
    by = buf[:1000] * 0.5
    ref = _np(ctx.source_sb(x, y, bx[:1000], by, sc.source, sc.lens_light))
    with pytest.raises(JtError) as e:
        ctx.source_sb(x, y, bx[:1000], by, sc.source, sc.lens_light, out=bx[1:1001])
    assert e.value.status == JT_EINVAL
    inplace = bx[:1000].clone()
    ctx.source_sb(x, y, inplace, by, sc.source, sc.lens_light, out=inplace)
    np.testing.assert_array_equal(_np(inplace), ref)


def test_invalid_arguments_raise_without_launch(ctx):
    from paper_2606_01547_amd import JtError
    from paper_2606_01547_amd._native import JT_EINVAL, JT_EUNSUPPORTED
    sc = W.config1_scene()
    x, y = W.random_points(10, 1.0, seed=0)
    with pytest.raises(JtError) as e:
        ctx.convolve(np.ones((8, 8), np.float32), np.ones((4, 4), np.float32))
    assert e.value.status == JT_EINVAL
    bad = W.Lens(sie=W.SIE(1.0, 0.0, 0.0, 0.0, 0.0))
    with pytest.raises(JtError) as e:
        ctx.deflection(x, y, bad)
    assert e.value.status == JT_EINVAL
    with pytest.raises(JtError):
        ctx.deflection(x, y, W.Lens(sie=W.SIE(1.0, 1.5, 0.0, 0.0, 0.0)))
    with pytest.raises(JtError):
        ctx.simulate_image(W.Grid(nx=0, ny=4, pixel_scale=0.05), sc.lens, sc.source)
    with pytest.raises(JtError):
        ctx.simulate_image(W.Grid(nx=4, ny=4, pixel_scale=0.05, supersample=17), sc.lens, sc.source)
    src = W.Sersic(amp=1.0, R_sersic=0.1, n_sersic=0.1, q=1.0, phi=0.0, cx=0.0, cy=0.0)
    with pytest.raises(JtError):
        ctx.source_sb(x, y, x, y, [src])
    with pytest.raises(JtError) as e:
        ctx.source_sb(x, y, x, y, [sc.source[0]] * 9)
    assert e.value.status == JT_EUNSUPPORTED
    with pytest.raises(JtError):
        ctx.upload_subhalos(W.NFWTable(np.zeros(3, np.float32), np.zeros(3, np.float32),
                                       np.array([0.1, 0.0, 0.1], np.float32), np.ones(3, np.float32)))
    with pytest.raises(JtError):
        ctx.release(987654321)
    # the context still works afterwards
    ax, ay = ctx.deflection(x, y, sc.lens)
    ex, ey = O.total_deflection(x, y, sc.lens)
    assert deflection_error(_np(ax), _np(ay), ex, ey) <= DEFLECTION_TOL
