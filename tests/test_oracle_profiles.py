"""Pins of the oracle's extra light profiles: Gaussian (total flux, centre
value, flux independent of q), core-Sersic (the Sersic as R_b -> 0, the inner
power-law slope -gamma), shapelets (phi_n against the Hermite closed forms of
low order, orthonormality of the 2-D basis by quadrature)."""
import math

import numpy as np
import pytest

import oracle as O


def _grid(half, n):
    g = (np.arange(n) + 0.5) * (2 * half / n) - half
    x, y = np.meshgrid(g, g)
    return x, y, (2 * half / n) ** 2


@pytest.mark.parametrize("q", [1.0, 0.6, 0.3])
def test_gaussian_total_flux_and_centre(q):
    x, y, da = _grid(3.0, 1200)
    I = O.gaussian(x, y, 7.5, 0.25, q, 0.7, 0.05, -0.1)
    assert abs(I.sum() * da - 7.5) < 1e-9
    c = O.gaussian(np.array([0.05]), np.array([-0.1]), 7.5, 0.25, q, 0.7, 0.05, -0.1)[0]
    assert abs(c - 7.5 / (2 * math.pi * 0.0625)) < 1e-12


def test_gaussian_is_isotropic_at_q_one():
    rng = np.random.default_rng(0)
    r = rng.uniform(0, 1, 50)
    a = rng.uniform(0, 2 * np.pi, 50)
    I = O.gaussian(r * np.cos(a), r * np.sin(a), 1.0, 0.3, 1.0, 1.1, 0.0, 0.0)
    np.testing.assert_allclose(I, np.exp(-r * r / 0.18) / (2 * math.pi * 0.09), rtol=1e-14)


def test_core_sersic_without_core_is_the_sersic():
    rng = np.random.default_rng(1)
    x, y = rng.uniform(-2, 2, (2, 200))
    a = O.core_sersic(x, y, 3.0, 0.6, 1e-9, 2.5, 0.4, 3.0, 0.7, 0.3, 0.1, 0.0)
    b = O.sersic(x, y, 3.0, 0.6, 2.5, 0.7, 0.3, 0.1, 0.0)
    np.testing.assert_allclose(a, b, rtol=1e-9)


@pytest.mark.parametrize("gamma", [0.2, 0.8, 1.5])
def test_core_sersic_inner_slope(gamma):
    Rb = 0.1
    r = np.array([1e-4, 1.01e-4]) * Rb
    I = O.core_sersic(r, np.zeros(2), 1.0, 1.0, Rb, 4.0, gamma, 2.0, 1.0, 0.0, 0.0, 0.0)
    slope = math.log(I[1] / I[0]) / math.log(r[1] / r[0])
    assert abs(slope + gamma) < 1e-3


def test_core_sersic_outside_the_break_approaches_the_sersic_shape():
    R = np.array([30.0, 60.0])
    a = O.core_sersic(R, np.zeros(2), 1.0, 5.0, 0.05, 2.0, 0.5, 4.0, 1.0, 0.0, 0.0, 0.0)
    b = O.sersic(R, np.zeros(2), 1.0, 5.0, 2.0, 1.0, 0.0, 0.0, 0.0)
    np.testing.assert_allclose(a, b, rtol=1e-7)


def test_shapelet_phi_low_orders():
    u = np.linspace(-3, 3, 41)
    g = np.exp(-u * u / 2) / math.pi ** 0.25
    np.testing.assert_allclose(O.shapelet_phi(0, u), g, rtol=1e-14)
    np.testing.assert_allclose(O.shapelet_phi(1, u), math.sqrt(2) * u * g, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(O.shapelet_phi(2, u), (2 * u * u - 1) / math.sqrt(2) * g, rtol=1e-13, atol=1e-15)


def test_shapelet_basis_is_orthonormal():
    n_max, beta = 4, 0.3
    x, y, da = _grid(3.0, 600)
    m = (n_max + 1) * (n_max + 2) // 2
    B = []
    for k in range(m):
        c = np.zeros(m)
        c[k] = 1.0
        B.append(O.shapelets(x, y, c, n_max, beta, 0.02, -0.03).ravel())
    B = np.array(B)
    G = B @ B.T * da
    np.testing.assert_allclose(G, np.eye(m), atol=1e-9)
    # the ordering: index of (n1, n2) = n (n + 1)/2 + n2
    c = np.zeros(m)
    c[O.shapelet_index(2, 1)] = 1.0
    u, v = (x - 0.02) / beta, (y + 0.03) / beta
    np.testing.assert_allclose(O.shapelets(x, y, c, n_max, beta, 0.02, -0.03),
                               O.shapelet_phi(2, u) * O.shapelet_phi(1, v) / beta, rtol=1e-13, atol=1e-15)
