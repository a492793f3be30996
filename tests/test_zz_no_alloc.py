"""The allocation-free fused simulation (jt_simulate_image_noalloc) against
jt_simulate_image, through the C ABI.

Both run the same kernels on the same inputs (the no-alloc call only keeps
its two intermediates -- the packed subhalo table and the unconvolved image --
in the library's static per-device scratch), so wherever jt_simulate_image
convolves directly the images must agree bit for bit; the bar of the image
parity tests (1e-4 floored relative error against the FP64 oracle) is checked
as well on the small case.  Two calls in a row with a smaller second input
show that the scratch's leftover contents from the first call do not leak into
the second.
"""
import dataclasses

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
    return t.cpu().numpy()


def _pair(ctx, sc, psf=True):
    p = sc.psf if psf else None
    a = _np(ctx.simulate_image(sc.grid, sc.lens, sc.source, sc.lens_light, p))
    b = _np(ctx.simulate_image(sc.grid, sc.lens, sc.source, sc.lens_light, p, noalloc=True))
    return a, b


def test_two_calls_second_smaller(ctx):
    """Headline image (200x200 px, s = 3, 10,000 NFW, 41x41 PSF), then a
    64x64 px, s = 1, 300-NFW image with an 11x11 PSF: each bit for bit the
    plain call's, the small one also within the oracle bar."""
    from paper_2606_01547_amd import _native
    big = W.config2_scene()
    assert _native.load_library().jt_convolve_auto_method(200, 200, 41) == 1
    a, b = _pair(ctx, big)
    assert np.isfinite(b).all() and np.abs(b).max() > 0
    np.testing.assert_array_equal(a, b)
    small = W.config2_scene(seed=77, n_sub=300, npix=64, supersample=1, psf_size=11)
    a, b = _pair(ctx, small)
    np.testing.assert_array_equal(a, b)
    ref = O.simulate_image(small)
    assert image_error(b.astype(np.float64), ref) <= IMAGE_TOL


def test_without_psf_and_truncated_subhalos(ctx):
    """No PSF (the fused kernel writes the caller's output; only the table
    uses the scratch), then TNFW subhalos (32-byte records) with a PSF."""
    sc = W.config2_scene(seed=5, n_sub=2000, npix=96, supersample=3, psf_size=21)
    a, b = _pair(ctx, sc, psf=False)
    np.testing.assert_array_equal(a, b)
    t = W.tnfw_scene(n_sub=1500, npix=80, supersample=3, psf_size=21)
    a, b = _pair(ctx, t)
    np.testing.assert_array_equal(a, b)


def test_resident_subhalo_table(ctx):
    """A resident subhalo handle: only the unconvolved image uses the scratch."""
    sc = W.config2_scene(seed=9, n_sub=4000, npix=120, supersample=3, psf_size=41)
    h = ctx.upload_subhalos(sc.lens.nfw)
    try:
        lens = dataclasses.replace(sc.lens, nfw=None)
        lens.subhalo_handle = h
        a = _np(ctx.simulate_image(sc.grid, sc.lens, sc.source, sc.lens_light, sc.psf))
        b = _np(ctx.simulate_image(sc.grid, lens, sc.source, sc.lens_light, sc.psf, noalloc=True))
        np.testing.assert_array_equal(a, b)
    finally:
        ctx.release(h)


def test_rejects_what_does_not_fit(ctx):
    """Argument errors are returned before any launch: an image whose
    unconvolved copy exceeds the 8 MiB scratch, and a PSF past the direct
    path's limit."""
    from paper_2606_01547_amd._native import JT_EUNSUPPORTED, JtError
    sc = W.config1_scene()
    g = dataclasses.replace(sc.grid, nx=1500, ny=1500)
    out = torch.empty((1500, 1500), dtype=torch.float32, device="cuda")
    with pytest.raises(JtError) as e:
        ctx.simulate_image(g, sc.lens, sc.source, sc.lens_light, sc.psf, out=out, noalloc=True)
    assert e.value.status == JT_EUNSUPPORTED and "static scratch" in str(e.value)
    big_psf = W.gaussian_psf(257, 2.0)
    with pytest.raises(JtError) as e:
        ctx.simulate_image(sc.grid, sc.lens, sc.source, sc.lens_light, big_psf, noalloc=True)
    assert e.value.status == JT_EUNSUPPORTED
    # still usable afterwards
    a, b = _pair(ctx, sc)
    np.testing.assert_array_equal(a, b)
