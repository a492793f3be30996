"""GPU parity of the batched forward, the chi^2 log-likelihood and its
hand-written adjoint against the FP64 oracle (autograd of the oracle forward).

Gradient bar per parameter group (macro; subhalo x; y; alpha_Rs):
  max |g_gpu - g_orc| / max(|g_orc|, 1e-3 max_group |g_orc|) <= 1e-3.
The GPU forward is FP32, so residuals carry ~1e-4 relative error and the
gradient inherits it; 1e-3 leaves a factor ~10.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import IMAGE_TOL, image_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GRAD_TOL = 1e-3


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


def _batch(scenes):
    from paper_2606_01547_amd.grad import DrawBatch, macro_row
    macro = np.stack([macro_row(s.lens, s.source, s.lens_light) for s in scenes])
    main = "epl" if getattr(scenes[0].lens, "epl", None) is not None else "sie"
    n = scenes[0].lens.nfw.n if scenes[0].lens.nfw is not None else 0
    if n == 0:
        return DrawBatch(macro, len(scenes[0].source), len(scenes[0].lens_light), main=main)
    st = lambda a: np.stack([getattr(s.lens.nfw, a) for s in scenes]).astype(np.float32)
    rt = st("r_trunc") if getattr(scenes[0].lens.nfw, "r_trunc", None) is not None else None
    return DrawBatch(macro, len(scenes[0].source), len(scenes[0].lens_light), st("x"), st("y"), st("Rs"),
                     st("alpha_Rs"), main=main, sub_r_trunc=rt)


def _group_err(g, e):
    g, e = np.asarray(g, np.float64), np.asarray(e, np.float64)
    den = np.maximum(np.abs(e), 1e-3 * np.abs(e).max())
    return float(np.max(np.abs(g - e) / den))


def _data(truth, seed=0):
    m = O.simulate_image(truth)
    d = W.noisy_image(m, seed=seed)
    w = (1.0 / O.noise_variance(d, 0.01, 1000.0)).astype(np.float32)
    return d, w


def test_batch_forward_equals_single_images(ctx):
    truth, draws = W.config4_draws(B=5, n_sub=300)
    out = _np(ctx.simulate_batch(truth.grid, _batch(draws), truth.psf))
    for b, sc in enumerate(draws):
        np.testing.assert_array_equal(out[b], _np(ctx.simulate_scene(sc)))
    assert image_error(out[2], O.simulate_image(draws[2])) <= IMAGE_TOL


def test_chi2_matches_oracle(ctx):
    truth, draws = W.config4_draws(B=4, n_sub=200)
    d, w = _data(truth)
    logL = _np(ctx.chi2(truth.grid, _batch(draws), d, w, truth.psf))
    models = _np(ctx.simulate_batch(truth.grid, _batch(draws), truth.psf))
    for b, sc in enumerate(draws):
        own = -0.5 * np.sum(w * (models[b] - d) ** 2)
        assert logL[b] == pytest.approx(own, rel=1e-5)          # the reduction itself
        ref = O.log_likelihood(O.simulate_image(sc), d, 0.01, 1000.0)
        assert logL[b] == pytest.approx(ref, rel=1e-3)           # FP32 model vs FP64 model


def _check_grad(ctx, truth, draws, d, w):
    logL, gm, gs = ctx.chi2_grad(truth.grid, _batch(draws), d, w, truth.psf)
    gm, gs = _np(gm), _np(gs)
    for b, sc in enumerate(draws):
        lo, em, es = O.chi2_gradient(sc, d.astype(np.float64), w.astype(np.float64))
        assert _group_err(gm[b], em) <= GRAD_TOL, (b, gm[b], em)
        if es.shape[0]:
            for col in range(3):
                assert _group_err(gs[b, :, col], es[:, col]) <= GRAD_TOL, (b, col)
        assert float(_np(logL)[b]) == pytest.approx(lo, rel=1e-3)


def test_chi2_grad_differentiation_case(ctx):
    """100x100 px, s = 1, 1000 NFW, 21x21 PSF (the benchmark's gradient shape)."""
    truth, draws = W.config4_draws(B=2)
    d, w = _data(truth, seed=1)
    _check_grad(ctx, truth, draws, d, w)


def test_chi2_grad_full_batch_sampled(ctx):
    """The benchmark's launch: 256 draws of the differentiation case in one
    call.  The last draw against the oracle; the first against the same draw
    computed alone, which runs with another wave split (8 instead of 1) and so
    groups its sub-pixels into other reduction blocks: equal to FP32 rounding."""
    truth, draws = W.config4_draws(B=256)
    d, w = _data(truth, seed=1)
    logL, gm, gs = ctx.chi2_grad(truth.grid, _batch(draws), d, w, truth.psf)
    gm, gs, logL = _np(gm), _np(gs), _np(logL)
    lo, em, es = O.chi2_gradient(draws[255], d.astype(np.float64), w.astype(np.float64))
    assert _group_err(gm[255], em) <= GRAD_TOL
    for col in range(3):
        assert _group_err(gs[255, :, col], es[:, col]) <= GRAD_TOL
    assert float(logL[255]) == pytest.approx(lo, rel=1e-3)
    # each entry sums 10^4 sub-pixel terms of both signs in FP32; another
    # grouping moves it by up to ~1e-5 of the group's largest (measured 1.2e-5)
    one = ctx.chi2_grad(truth.grid, _batch(draws[:1]), d, w, truth.psf)
    assert _group_err(gm[0], _np(one[1])[0]) <= 1e-4
    for col in range(3):
        assert _group_err(gs[0, :, col], _np(one[2])[0, :, col]) <= 1e-4
    assert np.all(np.isfinite(gm)) and np.all(np.isfinite(gs))


def test_adjoint_matches_central_differences_of_the_gpu_forward(ctx):
    """The differentiation case's macro gradient against central differences
    (h = 1e-4, relative) of jt_chi2 itself: the 28 perturbed draws in one
    batched forward.  FP32 model rounding puts ~1e-3 of noise on the
    differences of the large components; small ones are compared against 2%
    of the largest."""
    from paper_2606_01547_amd.grad import DrawBatch
    truth, draws = W.config4_draws(B=1)
    d, w = _data(truth, seed=3)
    base = _batch(draws)
    _, gm, _ = ctx.chi2_grad(truth.grid, base, d, w, truth.psf)
    g = _np(gm)[0]
    P = base.macro.shape[1]
    rows, hs = [], []
    for k in range(P):
        h = 1e-4 * max(abs(base.macro[0, k]), 0.1)
        for sgn in (1.0, -1.0):
            r = base.macro[0].copy()
            r[k] += sgn * h
            rows.append(r)
        hs.append(h)
    rep = lambda a: np.repeat(np.asarray(a), 2 * P, axis=0)
    pert = DrawBatch(np.stack(rows), base.n_src, base.n_ll, rep(base.sub_x), rep(base.sub_y), rep(base.sub_Rs),
                     rep(base.sub_alpha_Rs))
    L = _np(ctx.chi2(truth.grid, pert, d, w, truth.psf))
    fd = np.array([(L[2 * k] - L[2 * k + 1]) / (2 * hs[k]) for k in range(P)])
    big = np.abs(g) > 0.05 * np.abs(g).max()
    assert big.sum() >= 4
    np.testing.assert_allclose(g[big], fd[big], rtol=1e-2)
    assert np.max(np.abs(g - fd)) <= 0.02 * np.abs(g).max()


def test_chi2_grad_supersampled_with_lens_light(ctx):
    grid = W.Grid(nx=37, ny=29, pixel_scale=0.09, x0=0.04, y0=-0.03, supersample=2)
    truth, draws = W.config4_draws(B=3, n_sub=150, grid=grid, lens_light=True, psf_size=7)
    d, w = _data(truth, seed=2)
    _check_grad(ctx, truth, draws, d, w)


def test_chi2_grad_without_subhalos_or_psf(ctx):
    grid = W.Grid(nx=31, ny=33, pixel_scale=0.1, supersample=3)
    truth, draws = W.config4_draws(B=2, n_sub=1, grid=grid)
    for sc in [truth] + draws:
        sc.lens.nfw = None
        sc.psf = None
    d, w = _data(truth, seed=3)
    logL, gm, gs = ctx.chi2_grad(truth.grid, _batch(draws), d, w, None)
    for b, sc in enumerate(draws):
        _, em, _ = O.chi2_gradient(sc, d.astype(np.float64), w.astype(np.float64))
        assert _group_err(_np(gm)[b], em) <= GRAD_TOL
    assert gs.numel() == 0


def test_gradient_is_zero_at_the_gpu_model(ctx):
    truth, draws = W.config4_draws(B=2, n_sub=100)
    m = ctx.simulate_batch(truth.grid, _batch(draws[:1]), truth.psf)[0]
    d = m.clone()
    w = torch.ones_like(m)
    logL, gm, gs = ctx.chi2_grad(truth.grid, _batch(draws[:1]), d, w, truth.psf)
    assert _np(logL)[0] == 0.0
    assert np.all(_np(gm) == 0.0) and np.all(_np(gs) == 0.0)


def test_gradient_deterministic_and_batch_independent(ctx):
    truth, draws = W.config4_draws(B=6, n_sub=400)
    d, w = _data(truth, seed=4)
    a = ctx.chi2_grad(truth.grid, _batch(draws), d, w, truth.psf)
    b = ctx.chi2_grad(truth.grid, _batch(draws), d, w, truth.psf)
    c = ctx.chi2_grad(truth.grid, _batch(draws[3:4]), d, w, truth.psf)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(_np(x), _np(y))
    np.testing.assert_array_equal(_np(a[1])[3], _np(c[1])[0])
    np.testing.assert_array_equal(_np(a[2])[3], _np(c[2])[0])


@pytest.mark.parametrize("n_sub,s,lens_light", [(400, 1, False), (150, 3, True), (0, 2, False)])
def test_kept_positions_give_the_recomputed_gradient_bit_for_bit(ctx, n_sub, s, lens_light):
    grid = W.Grid(nx=52, ny=47, pixel_scale=0.08, supersample=s)
    truth, draws = W.config4_draws(B=5, n_sub=max(n_sub, 1), grid=grid, lens_light=lens_light)
    if n_sub == 0:
        for sc in [truth] + draws:
            sc.lens.nfw = None
    d, w = _data(truth, seed=6)
    a = ctx.chi2_grad(truth.grid, _batch(draws), d, w, truth.psf)
    b = ctx.chi2_grad(truth.grid, _batch(draws), d, w, truth.psf, keep_positions=True)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(_np(x), _np(y))


def test_autograd_function_backward_is_the_adjoint(ctx):
    from paper_2606_01547_amd.grad import chi2_loglike
    truth, draws = W.config4_draws(B=3, n_sub=120)
    d, w = _data(truth, seed=5)
    bt = _batch(draws)
    macro = torch.tensor(bt.macro, dtype=torch.float64, requires_grad=True)
    dev = torch.device("cuda", 0)
    sx = torch.tensor(bt.sub_x, device=dev, requires_grad=True)
    sy = torch.tensor(bt.sub_y, device=dev, requires_grad=True)
    sa = torch.tensor(bt.sub_alpha_Rs, device=dev, requires_grad=True)
    srs = torch.tensor(bt.sub_Rs, device=dev)
    logL = chi2_loglike(ctx, truth.grid, macro, sx, sy, srs, sa, bt.n_src, bt.n_ll, d, w, truth.psf)
    scale = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device=logL.device)
    (logL * scale).sum().backward()
    _, gm, gs = ctx.chi2_grad(truth.grid, bt, d, w, truth.psf)
    gm, gs = _np(gm), _np(gs)
    s = np.array([1.0, -2.0, 0.5])
    np.testing.assert_allclose(macro.grad.numpy(), gm * s[:, None], rtol=1e-6)
    np.testing.assert_allclose(_np(sx.grad), gs[..., 0] * s[:, None], rtol=1e-6)
    np.testing.assert_allclose(_np(sa.grad), gs[..., 2] * s[:, None], rtol=1e-6)


def test_batch_output_overlapping_the_psf_is_rejected(ctx):
    from paper_2606_01547_amd import JtError
    from paper_2606_01547_amd._native import JT_EINVAL
    grid = W.Grid(nx=16, ny=16, pixel_scale=0.1)
    truth, draws = W.config4_draws(B=2, n_sub=10, grid=grid, psf_size=5)
    buf = torch.zeros(2 * 256 + 25, device="cuda")
    buf[2 * 256 - 10:2 * 256 + 15] = torch.from_numpy(truth.psf.ravel().astype(np.float32)).cuda()
    with pytest.raises(JtError) as e:
        ctx.simulate_batch(grid, _batch(draws), buf[2 * 256 - 10:2 * 256 + 15].view(5, 5),
                           out=buf[:512].view(2, 16, 16))
    assert e.value.status == JT_EINVAL


def test_gradient_argument_errors(ctx):
    from paper_2606_01547_amd import JtError
    from paper_2606_01547_amd._native import JT_EUNSUPPORTED
    grid = W.Grid(nx=16, ny=16, pixel_scale=0.1)
    truth, draws = W.config4_draws(B=1, n_sub=10, grid=grid, lens_light=True)
    for sc in draws:
        sc.source = sc.source * 3
    d, w = np.zeros((16, 16), np.float32), np.ones((16, 16), np.float32)
    with pytest.raises(JtError) as e:
        ctx.chi2_grad(grid, _batch(draws), d, w, truth.psf)
    assert e.value.status == JT_EUNSUPPORTED
    with pytest.raises(JtError):
        ctx.chi2(grid, _batch(draws), d, w, np.ones((4, 4), np.float32))


# ------------------------------------- EPL main deflector, truncated subhalos
@pytest.mark.parametrize("epl,tnfw", [(True, False), (False, True), (True, True)])
def test_chi2_grad_epl_and_truncated_subhalos(ctx, epl, tnfw):
    """The adjoint with an EPL main deflector (its six partials, the slope
    included) and/or truncated subhalos, against the oracle's autograd
    gradient: 48x44 px, s = 2, 300 subhalos, 7x7 PSF, 3 draws."""
    grid = W.Grid(nx=48, ny=44, pixel_scale=0.1, x0=0.02, y0=-0.03, supersample=2)
    truth, draws = W.config4_profile_draws(B=3, n_sub=300, grid=grid, epl=epl, tnfw=tnfw)
    d, w = _data(truth, seed=8)
    b = _batch(draws)
    assert b.main == ("epl" if epl else "sie") and (b.sub_r_trunc is not None) == tnfw
    _check_grad(ctx, truth, draws, d, w)


def test_epl_tnfw_batch_forward_equals_single_images(ctx):
    grid = W.Grid(nx=40, ny=36, pixel_scale=0.1, supersample=3)
    truth, draws = W.config4_profile_draws(B=4, n_sub=200, grid=grid, epl=True, tnfw=True)
    out = _np(ctx.simulate_batch(truth.grid, _batch(draws), truth.psf))
    for k, sc in enumerate(draws):
        np.testing.assert_array_equal(out[k], _np(ctx.simulate_scene(sc)))
    assert image_error(out[1], O.simulate_image(draws[1])) <= IMAGE_TOL


def test_epl_tnfw_kept_positions_bit_for_bit(ctx):
    grid = W.Grid(nx=44, ny=41, pixel_scale=0.09, supersample=2)
    truth, draws = W.config4_profile_draws(B=4, n_sub=250, grid=grid, epl=True, tnfw=True)
    d, w = _data(truth, seed=9)
    a = ctx.chi2_grad(truth.grid, _batch(draws), d, w, truth.psf)
    b = ctx.chi2_grad(truth.grid, _batch(draws), d, w, truth.psf, keep_positions=True)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(_np(x), _np(y))


def test_truncated_near_pairs_at_the_grid_edges(ctx):
    """The truncated subhalos' near pairs (the general form, a wave per subhalo
    over its box of the sub-pixel grid) against the oracle's autograd gradient,
    with subhalos placed where that box is clamped or empty: next to a
    sub-pixel centre, on the left edge, centred outside a corner with its near
    region reaching into the grid, far outside it, and one whose near region
    covers the whole grid; the other subhalos as drawn.  42x38 px, s = 2."""
    grid = W.Grid(nx=42, ny=38, pixel_scale=0.1, x0=0.01, y0=-0.02, supersample=2)
    truth, draws = W.config4_profile_draws(B=2, n_sub=60, grid=grid, epl=False, tnfw=True)
    d_px, s = grid.pixel_scale, grid.supersample
    ox, oy = grid.x0 - d_px * grid.nx / 2, grid.y0 - d_px * grid.ny / 2
    step = d_px / s
    for sc in draws:
        t = sc.lens.nfw
        place = [(ox + step * (11 + 0.5) + 1e-3 * step, oy + step * (9 + 0.5), 0.05, 10.0),   # by a centre
                 (ox + 0.3 * step, oy + 0.4 * (grid.ny * d_px), 0.08, 12.0),                # left edge
                 (ox - 0.15, oy - 0.12, 0.06, 20.0),                                          # outside a corner
                 (ox - 50.0, oy + 1.0, 0.05, 10.0),                                           # far outside
                 (grid.x0 + 0.3, grid.y0 - 0.2, 0.3, 30.0)]                                   # covers the grid
        for i, (x, y, rs, tau) in enumerate(place):
            t.x[i], t.y[i], t.Rs[i], t.r_trunc[i] = x, y, rs, tau * rs
    # near regions: rho = max(0.75 tau, 1.5) Rs
    assert 0.75 * 30.0 * 0.3 > np.hypot(grid.nx * d_px / 2 + 0.3, grid.ny * d_px / 2 + 0.2)
    d, w = _data(truth, seed=12)
    _check_grad(ctx, truth, draws, d, w)
