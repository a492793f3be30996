"""The continuous-batching server on the GPU: every request's image is
bitwise the same as the same request simulated alone (fixed summation order;
each convolution takes the launch shape and LDS row chunk the image alone
would get), and matches the oracle; requests of very different sizes share
launches and streams.  jt_simulate_image may pick the FFT convolution for
large images with large kernels, where the server convolves directly: those
agree to the image tolerance only, so the bitwise comparisons here stay on
sizes whose automatic choice is the direct path (asserted)."""
import time

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


def _requests(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        npx = int(rng.choice([17, 32, 50, 64, 100]))
        s = int(rng.choice([1, 3]))
        nsub = int(rng.choice([0, 5, 300, 2000]))
        k = int(rng.choice([0, 11, 21]))
        sc = W.config2_scene(seed=seed * 1000 + i, n_sub=max(nsub, 1), npix=npx, supersample=s,
                             psf_size=k if k else 11)
        if nsub == 0:
            sc.lens.nfw = None
        if k == 0:
            sc.psf = None
        out.append(sc)
    return out


def _serve(ctx, scenes, gaps=None, **cfg):
    from paper_2606_01547_amd import Server
    srv = Server(ctx, **cfg)
    handles, outs, tickets = [], [], []
    for i, sc in enumerate(scenes):
        hs = ctx.upload_subhalos(sc.lens.nfw) if sc.lens.nfw is not None else 0
        hp = ctx.upload_psf(sc.psf) if sc.psf is not None else 0
        handles += [h for h in (hs, hp) if h]
        o = torch.full((sc.grid.ny, sc.grid.nx), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        outs.append(o)
        tickets.append(srv.submit(sc.grid, sc.lens, sc.source, sc.lens_light, out=o, subhalo_handle=hs,
                                  psf_handle=hp))
        if gaps is not None:
            time.sleep(gaps[i])
    lat = [srv.wait(t, timeout=60.0) for t in tickets]
    stats = srv.stats()
    srv.close()
    for h in handles:
        ctx.release(h)
    return outs, lat, stats


def test_mixed_stream_equals_single_requests(ctx):
    scenes = _requests(40, seed=7)
    gaps = np.random.default_rng(1).exponential(2e-4, len(scenes))
    outs, lat, st = _serve(ctx, scenes, gaps, hbm_budget_bytes=256 << 20, max_batch_images=16,
                           max_batch_pairs=5e8, max_inflight_batches=3, n_streams=3)
    assert st["completed"] == 40 and st["arena_in_use"] == 0 and st["failed"] == 0
    assert min(lat) > 0
    _assert_direct(scenes)
    for sc, o in zip(scenes, outs):
        alone = ctx.simulate_scene(sc)
        np.testing.assert_array_equal(_np(o), _np(alone))
    for sc, o in list(zip(scenes, outs))[:6]:
        assert image_error(_np(o), O.simulate_image(sc)) <= IMAGE_TOL


def _assert_direct(scenes):
    from paper_2606_01547_amd import convolve_auto_method
    for sc in scenes:
        if sc.psf is not None:
            k = sc.psf.shape[0]
            assert convolve_auto_method(sc.grid.nx, sc.grid.ny, k) == 1, (sc.grid.nx, k)


def test_mixed_psf_batch_equals_single_requests(ctx):
    """An 11x11, a 21x21 and a 41x41 PSF request, two 400x400 ones, a 500x500
    and a 1000x1000 one share one batch: their convolutions take all three
    launch shapes of the direct path (one 16-column group split over eight
    waves, two groups of two waves, four groups of one wave; the server
    launches each shape's tiles together) and different LDS row chunks; every
    image is still the request alone bit for bit.  A long first request on
    the single in-flight slot makes the rest queue and launch together."""
    first = W.config2_scene(seed=51, n_sub=20000, npix=400, supersample=3, psf_size=21)
    rest = [W.config2_scene(seed=52, n_sub=100, npix=64, supersample=1, psf_size=11),
            W.config2_scene(seed=53, n_sub=300, npix=100, supersample=3, psf_size=21),
            W.config2_scene(seed=54, n_sub=200, npix=400, supersample=1, psf_size=21),
            W.config2_scene(seed=55, n_sub=50, npix=400, supersample=1, psf_size=21),
            W.config2_scene(seed=56, n_sub=500, npix=200, supersample=1, psf_size=41),
            W.config2_scene(seed=57, n_sub=50, npix=500, supersample=1, psf_size=21),
            W.config2_scene(seed=58, n_sub=30, npix=1000, supersample=1, psf_size=11)]
    scenes = [first] + rest
    _assert_direct(scenes)
    from paper_2606_01547_amd import Server
    # everything resident and allocated before the first submission, so that
    # no device synchronisation separates the submissions
    hs = [ctx.upload_subhalos(sc.lens.nfw) for sc in scenes]
    hp = [ctx.upload_psf(sc.psf) for sc in scenes]
    outs = [torch.full((sc.grid.ny, sc.grid.nx), float("nan"), dtype=torch.float32, device="cuda") for sc in scenes]
    torch.cuda.synchronize()
    srv = Server(ctx, hbm_budget_bytes=512 << 20, max_batch_images=16, max_batch_pairs=1e11,
                 max_inflight_batches=1, n_streams=1)
    tickets = [srv.submit(sc.grid, sc.lens, sc.source, sc.lens_light, out=o, subhalo_handle=h, psf_handle=p)
               for sc, o, h, p in zip(scenes, outs, hs, hp)]
    for t in tickets:
        srv.wait(t, timeout=60.0)
    st = srv.stats()
    srv.close()
    for h in hs + hp:
        ctx.release(h)
    assert st["completed"] == len(scenes) and st["failed"] == 0
    assert st["batches"] == 2, st                     # the long request, then the other seven at once
    for sc, o in zip(scenes, outs):
        np.testing.assert_array_equal(_np(o), _np(ctx.simulate_scene(sc)))
    assert image_error(_np(outs[1]), O.simulate_image(rest[0])) <= IMAGE_TOL


def test_large_request_in_the_mix(ctx):
    big = W.config2_scene()                                  # 200x200, s = 3, 10k NFW, 41x41 PSF
    small = _requests(12, seed=9)
    scenes = small[:6] + [big] + small[6:]
    outs, lat, st = _serve(ctx, scenes, None, hbm_budget_bytes=512 << 20, max_batch_images=8,
                           max_batch_pairs=2e8, max_inflight_batches=4, n_streams=4)
    assert st["completed"] == len(scenes)
    np.testing.assert_array_equal(_np(outs[6]), _np(ctx.simulate_scene(big)))
    for sc, o in zip(scenes, outs):
        np.testing.assert_array_equal(_np(o), _np(ctx.simulate_scene(sc)))


def test_chunked_requests_equal_single_requests(ctx):
    """Requests over the work cap run as chunks of pixel blocks on one stream;
    the image (with and without a PSF) is the same as the request alone."""
    big1 = W.config2_scene(seed=21, n_sub=2000, npix=500, supersample=3, psf_size=21)   # 8929 blocks
    big2 = W.config2_scene(seed=22, n_sub=3000, npix=520, supersample=3)                # 9658 blocks
    big2.psf = None
    small = _requests(6, seed=13)
    scenes = [big1] + small[:3] + [big2] + small[3:]
    outs, lat, st = _serve(ctx, scenes, None, hbm_budget_bytes=256 << 20, max_batch_images=8,
                           max_batch_pairs=2e7, max_inflight_batches=4, n_streams=4)
    assert st["completed"] == len(scenes) and st["failed"] == 0 and st["arena_in_use"] == 0
    assert st["batches"] >= 3 + 1 + 3                # chunks of >= 2048 blocks, one convolution
    for sc, o in zip(scenes, outs):
        np.testing.assert_array_equal(_np(o), _np(ctx.simulate_scene(sc)))


def test_epl_requests_equal_single_requests(ctx):
    """Requests with an elliptical power-law main deflector batch beside SIE
    requests and give the same image as alone."""
    epl = [W.epl_scene(seed=30 + i, n_sub=n, npix=p, supersample=s, psf_size=21)
           for i, (n, p, s) in enumerate([(1, 40, 3), (500, 64, 1), (2000, 50, 3)])]
    scenes = _requests(4, seed=15)
    scenes = scenes[:2] + epl + scenes[2:]
    outs, lat, st = _serve(ctx, scenes, None, hbm_budget_bytes=256 << 20, max_batch_images=8,
                           max_batch_pairs=5e8, max_inflight_batches=3, n_streams=2)
    assert st["completed"] == len(scenes) and st["failed"] == 0
    for sc, o in zip(scenes, outs):
        np.testing.assert_array_equal(_np(o), _np(ctx.simulate_scene(sc)))
    assert image_error(_np(outs[2]), O.simulate_image(epl[0])) <= IMAGE_TOL


def test_truncated_subhalo_requests_equal_single_requests(ctx):
    """Requests with resident truncated-NFW tables are served beside NFW ones
    (never in the same launch), one of them in chunks over the work cap, and
    each image is the same as the request alone."""
    tnfw = [W.tnfw_scene(seed=40 + i, n_sub=n, npix=p, supersample=s, psf_size=21)
            for i, (n, p, s) in enumerate([(50, 20, 1), (300, 64, 3), (1000, 50, 1)])]
    big = W.tnfw_scene(seed=45, n_sub=200, npix=400, supersample=3, psf_size=21)    # 5715 blocks: chunked
    scenes = _requests(5, seed=17)
    scenes = scenes[:1] + tnfw[:2] + scenes[1:3] + [big, tnfw[2]] + scenes[3:]
    outs, lat, st = _serve(ctx, scenes, None, hbm_budget_bytes=256 << 20, max_batch_images=8,
                           max_batch_pairs=2e8, max_inflight_batches=3, n_streams=3)
    assert st["completed"] == len(scenes) and st["failed"] == 0 and st["arena_in_use"] == 0
    for sc, o in zip(scenes, outs):
        np.testing.assert_array_equal(_np(o), _np(ctx.simulate_scene(sc)))
    assert image_error(_np(outs[1]), O.simulate_image(tnfw[0])) <= IMAGE_TOL


def test_tight_arena_serialises_but_completes(ctx):
    scenes = _requests(10, seed=11)
    outs, lat, st = _serve(ctx, scenes, None, hbm_budget_bytes=1 << 20, max_batch_images=4,
                           max_batch_pairs=1e12, max_inflight_batches=2, n_streams=2)
    assert st["completed"] == 10 and st["arena_peak"] <= (1 << 20)
    for sc, o in zip(scenes, outs):
        np.testing.assert_array_equal(_np(o), _np(ctx.simulate_scene(sc)))
