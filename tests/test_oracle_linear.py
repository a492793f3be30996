"""Pins of the oracle's linear amplitude solver: the image is linear in the
amplitudes (the basis images sum back to the simulated image), noise-free
data returns the true amplitudes, the weighted residual is orthogonal to
every basis image, and the solution maximises the log-likelihood."""
import numpy as np

import oracle as O
import workloads as W


def _scene():
    sc = W.config2_scene(n_sub=40, npix=36, supersample=2, psf_size=11)
    sc.source.append(W.Sersic(amp=2.5, R_sersic=0.3, n_sersic=1.5, q=0.7, phi=0.4, cx=0.2, cy=-0.1))
    return sc


def test_basis_images_sum_to_the_image():
    sc = _scene()
    B = O.basis_images(sc)
    amps = [c.amp for c in sc.source] + [c.amp for c in sc.lens_light]
    assert B.shape == (4, 36, 36)
    np.testing.assert_allclose(np.tensordot(amps, B, 1), O.simulate_image(sc), rtol=1e-12, atol=1e-14)


def test_noise_free_data_returns_the_amplitudes():
    sc = _scene()
    d = O.simulate_image(sc)
    w = O.noise_variance(d, 0.01, 1000.0) ** -1
    amps, model, logL = O.linear_amplitudes(sc, d, w)
    truth = [c.amp for c in sc.source] + [c.amp for c in sc.lens_light]
    np.testing.assert_allclose(amps, truth, rtol=1e-9)
    np.testing.assert_allclose(model, d, rtol=1e-9, atol=1e-12)
    assert abs(logL) < 1e-12


def test_weighted_residual_is_orthogonal_to_the_basis():
    sc = _scene()
    d = W.noisy_image(O.simulate_image(sc), seed=3).astype(np.float64)
    w = O.noise_variance(d, 0.01, 1000.0) ** -1
    B = O.basis_images(sc)
    amps, model, _ = O.linear_amplitudes(sc, d, w, basis=B)
    r = w * (d - model)
    for b in B:
        assert abs(np.sum(b * r)) <= 1e-9 * np.sum(np.abs(b * w * d))


def test_solution_maximises_the_likelihood():
    sc = _scene()
    d = W.noisy_image(O.simulate_image(sc), seed=4).astype(np.float64)
    w = O.noise_variance(d, 0.01, 1000.0) ** -1
    B = O.basis_images(sc)
    amps, _, logL = O.linear_amplitudes(sc, d, w, basis=B)
    ll = lambda a: -0.5 * np.sum(w * (d - np.tensordot(a, B, 1)) ** 2)
    assert abs(ll(amps) - logL) <= 1e-9 * abs(logL)
    for j in range(len(amps)):
        for s in (-1e-3, 1e-3):
            a = amps.copy()
            a[j] += s * max(1.0, abs(a[j]))
            assert ll(a) < logL
