"""GPU parity of the extra light profiles (Gaussian, multi-Gaussian,
core-Sersic, shapelets) against the oracle: point evaluation through
jt_source_sb, full images through jt_simulate_image, and the server."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import IMAGE_TOL, image_error

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


def _shapelets(n_max, seed, beta=0.15, cx=0.05, cy=-0.03):
    rng = np.random.default_rng(seed)
    m = (n_max + 1) * (n_max + 2) // 2
    return W.Shapelets(n_max=n_max, beta=beta, cx=cx, cy=cy, coeff=rng.normal(0, 1, m) / (1 + np.arange(m)))


def _gaussians(k, elliptical, seed):
    rng = np.random.default_rng(seed)
    return [W.Gaussian(amp=float(rng.uniform(1, 5)), sigma=float(rng.uniform(0.05, 0.4)),
                       q=float(rng.uniform(0.4, 1.0)) if elliptical else 1.0, phi=float(rng.uniform(0, np.pi)),
                       cx=0.02, cy=-0.01) for _ in range(k)]


CORE = W.CoreSersic(amp=2.0, R_sersic=0.5, R_b=0.08, n_sersic=4.0, gamma=0.3, alpha=3.0, q=0.75, phi=0.6,
                    cx=-0.03, cy=0.02)


@pytest.mark.parametrize("case", ["gauss", "gauss_ellipse", "multi_gauss5", "multi_gauss5_ellipse", "core",
                                  "shapelets6", "shapelets10", "mixed"])
def test_source_sb_extra_profiles(ctx, case):
    comps = {"gauss": _gaussians(1, False, 1), "gauss_ellipse": _gaussians(1, True, 2),
             "multi_gauss5": _gaussians(5, False, 3), "multi_gauss5_ellipse": _gaussians(5, True, 4),
             "core": [CORE], "shapelets6": [_shapelets(6, 5)], "shapelets10": [_shapelets(10, 6)],
             "mixed": [W.Sersic(3.0, 0.3, 2.0, 0.8, 0.2, 0.0, 0.0), _shapelets(4, 7)] + _gaussians(2, True, 8) +
                      [CORE]}[case]
    x, y = W.random_points(5000, 1.2, seed=11)
    bx, by = W.random_points(5000, 1.2, seed=12)
    # positive profiles hold 1e-5; a shapelet set is a signed sum whose FP32
    # round-off near its zero crossings is measured against the image bar
    tol = IMAGE_TOL if case.startswith("shapelets") or case == "mixed" else 1e-5
    for src, ll in ((comps, []), ([], comps)):
        got = _np(ctx.source_sb(x, y, bx, by, src, ll))
        ref = O.surface_brightness(x, y, bx, by, src, ll)
        assert image_error(got, ref) <= tol, case


def test_core_sersic_at_its_centre(ctx):
    c = W.CoreSersic(amp=1.0, R_sersic=0.5, R_b=0.1, n_sersic=3.0, gamma=0.5, alpha=2.0, q=1.0, phi=0.0,
                     cx=0.25, cy=-0.125)
    x = np.array([0.25, 0.25], dtype=np.float32)
    y = np.array([-0.125, -0.12], dtype=np.float32)
    got = _np(ctx.source_sb(x, y, x, y, [c], []))
    ref = O.surface_brightness(x, y, x, y, [c], [])
    np.testing.assert_allclose(got, ref, rtol=2e-5)


def test_simulate_with_extra_profiles(ctx):
    sc = W.config2_scene(n_sub=1500, npix=40, supersample=3, psf_size=21)
    sc.grid = W.Grid(nx=40, ny=34, pixel_scale=0.05, x0=0.02, y0=-0.03, supersample=3)
    sc.source = [sc.source[0], _shapelets(8, 9, beta=0.1)] + _gaussians(2, True, 10)
    sc.lens_light = [CORE] + _gaussians(3, False, 11)
    got = _np(ctx.simulate_scene(sc))
    assert image_error(got, O.simulate_image(sc)) <= IMAGE_TOL


def test_every_profile_at_once(ctx):
    """EPL main deflector, shear, truncated subhalos, Sersic, core-Sersic,
    Gaussian and shapelet light in one image, against the oracle."""
    sc = W.epl_scene(seed=77, n_sub=800, npix=36, supersample=3, psf_size=15)
    sc.grid = W.Grid(nx=36, ny=31, pixel_scale=0.06, x0=0.01, y0=-0.02, supersample=3)
    rng = np.random.default_rng(78)
    sc.lens.nfw.r_trunc = (10.0 ** rng.uniform(0.5, 1.5, sc.lens.nfw.n) * sc.lens.nfw.Rs).astype(np.float32)
    sc.source = [sc.source[0], _shapelets(5, 79, beta=0.1)] + _gaussians(2, True, 80)
    sc.lens_light = [CORE] + _gaussians(1, False, 81)
    got = _np(ctx.simulate_scene(sc))
    assert image_error(got, O.simulate_image(sc)) <= IMAGE_TOL


@pytest.mark.parametrize("make", [W.config2_scene, W.tnfw_scene], ids=["nfw", "tnfw"])
def test_server_serves_extra_profiles(ctx, make):
    from paper_2606_01547_amd import Server
    scenes = []
    for i in range(4):
        sc = make(seed=40 + i, n_sub=200, npix=32, supersample=1 + 2 * (i % 2), psf_size=11)
        sc.source.append(_shapelets(3 + i, 20 + i, beta=0.12))
        sc.lens_light = _gaussians(2, True, 30 + i)
        scenes.append(sc)
    srv = Server(ctx, hbm_budget_bytes=64 << 20, max_batch_images=4, max_batch_pairs=1e8, max_inflight_batches=2,
                 n_streams=2)
    outs, hs = [], []
    for sc in scenes:
        h = ctx.upload_subhalos(sc.lens.nfw)
        hp = ctx.upload_psf(sc.psf)
        hs += [h, hp]
        o = torch.empty((sc.grid.ny, sc.grid.nx), dtype=torch.float32, device="cuda")
        outs.append((o, srv.submit(sc.grid, sc.lens, sc.source, sc.lens_light, out=o, subhalo_handle=h,
                                   psf_handle=hp)))
    for o, t in outs:
        srv.wait(t, timeout=60.0)
    srv.close()
    for h in hs:
        ctx.release(h)
    for sc, (o, _) in zip(scenes, outs):
        np.testing.assert_array_equal(_np(o), _np(ctx.simulate_scene(sc)))


def test_extra_profiles_reject_bad_parameters(ctx):
    from paper_2606_01547_amd import JtError
    x, y = W.random_points(8, 1.0, seed=1)
    bad = [W.Gaussian(1.0, 0.0, 1.0, 0, 0, 0), W.Gaussian(1.0, 0.1, 1.5, 0, 0, 0),
           W.CoreSersic(1.0, 0.5, 0.1, 3.0, 2.5, 2.0, 1.0, 0, 0, 0),
           W.CoreSersic(1.0, 0.5, 0.0, 3.0, 0.5, 2.0, 1.0, 0, 0, 0),
           W.Shapelets(11, 0.1, 0, 0, np.ones(78)), W.Shapelets(2, -0.1, 0, 0, np.ones(6))]
    for c in bad:
        with pytest.raises(JtError):
            ctx.source_sb(x, y, x, y, [c], [])
    with pytest.raises(JtError):
        ctx.source_sb(x, y, x, y, _gaussians(9, False, 1), [])
    sc = W.config1_scene()
    d = np.zeros((sc.grid.ny, sc.grid.nx), np.float32)
    with pytest.raises(JtError):
        ctx.linear_amplitudes(sc.grid, sc.lens, sc.source + _gaussians(1, False, 2), [], d, d + 1, psf=sc.psf)
