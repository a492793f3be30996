"""The seeded input generators: reproducible, FP32-exact, within their priors."""
import math

import numpy as np

import workloads as W


def _is_f32(v):
    return float(np.float32(v)) == v


def test_generators_are_deterministic_and_fp32():
    a = W.config2_scene(n_sub=200)
    b = W.config2_scene(n_sub=200)
    np.testing.assert_array_equal(a.lens.nfw.x, b.lens.nfw.x)
    np.testing.assert_array_equal(a.psf, b.psf)
    assert a.lens.sie == b.lens.sie
    for v in (a.lens.sie.theta_E, a.lens.sie.q, a.lens.sie.phi, a.lens.shear.gamma1,
              a.source[0].R_sersic, a.lens_light[0].n_sersic):
        assert _is_f32(v)
    assert a.lens.nfw.x.dtype == np.float32 and a.psf.dtype == np.float32


def test_priors_and_shapes():
    sc = W.config2_scene()
    s = sc.lens.sie
    assert 0.8 <= s.theta_E <= 1.5 and 0.6 <= s.q <= 1.0 and 0.0 <= s.phi < math.pi
    n = sc.lens.nfw
    assert n.n == 10000
    r = np.hypot(n.x - s.cx, n.y - s.cy)
    assert r.max() <= 3.0 + 1e-5
    assert 0.0115 < n.Rs.min() and n.Rs.max() < 0.245
    assert sc.psf.shape == (41, 41) and abs(float(sc.psf.sum(dtype=np.float64)) - 1) < 1e-6
    assert (sc.psf >= 0).all()
    assert sc.grid.nx == 200 and sc.grid.supersample == 3
    assert len(sc.source) == 2 and len(sc.lens_light) == 1


def test_config1_gaussian_psf_truncation():
    sc = W.config1_scene()
    assert sc.psf.shape == (11, 11)
    # sigma = 2 px / 2.3548 = 0.8493 px; truncation at 5 sigma = 4.25 px zeroes the corners
    assert sc.psf[0, 0] == 0.0 and sc.psf[5, 0] == 0.0 and sc.psf[5, 1] > 0.0
    np.testing.assert_allclose(sc.psf, sc.psf.T)


def test_nfw_mass_mapping_monotone():
    rs, ars = W.nfw_params_from_mass(np.logspace(6, 10, 9))
    assert np.all(np.diff(rs) > 0) and np.all(np.diff(ars) > 0)


def test_request_stream_mix():
    reqs = W.config3_requests(n_requests=24)
    sizes = {r.grid.nx for r in reqs}
    assert sizes <= {64, 100, 200, 400}
    assert all(0 <= (r.lens.nfw.n) <= 20000 for r in reqs)
    assert {r.psf.shape[0] for r in reqs} <= {21, 41}
