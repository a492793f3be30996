"""The stored oracle image of the headline workload (tests/golden/c2_headline.npz,
written by tests/golden/make_c2.py from the oracle alone) is still what the
oracle computes: checksums, a sample of pixels recomputed one by one (the
brightest among them), and the convolved image from the unconvolved one."""
import hashlib
import os

import numpy as np

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load():
    z = np.load(os.path.join(GOLDEN, "c2_headline.npz"))
    return z["unconvolved"], z["convolved"]


def test_golden_checksums():
    un, conv = _load()
    want = dict(line.split() for line in open(os.path.join(GOLDEN, "c2_headline.sha256")))
    assert hashlib.sha256(un.tobytes()).hexdigest() == want["unconvolved"]
    assert hashlib.sha256(conv.tobytes()).hexdigest() == want["convolved"]
    assert un.shape == conv.shape == (200, 200) and un.dtype == conv.dtype == np.float64


def test_golden_pixels_recomputed_by_the_oracle():
    un, conv = _load()
    sc = W.config2_scene()
    g = sc.grid
    top = np.argsort(un.reshape(-1))[-3:]
    rows = np.concatenate([[0, 199, 57, 140], top // 200])
    cols = np.concatenate([[0, 199, 131, 23], top % 200])
    tx, ty = O.subpixel_coords(g.nx, g.ny, g.pixel_scale, g.x0, g.y0, g.supersample)
    tx, ty = tx[rows, cols], ty[rows, cols]
    bx, by = O.ray_shoot(tx, ty, sc.lens)
    sb = O.surface_brightness(tx, ty, bx, by, sc.source, sc.lens_light, sc.bn_exact)
    ref = g.pixel_scale ** 2 * sb.mean(axis=(-2, -1))
    np.testing.assert_allclose(un[rows, cols], ref, rtol=1e-12, atol=0)
    np.testing.assert_allclose(conv, O.convolve_same(un, sc.psf), rtol=1e-12, atol=1e-15 * np.abs(conv).max())
