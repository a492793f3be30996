"""Pins of the oracle's image likelihood (`log_likelihood`, `noise_variance`).

The paper names log-likelihood choices among its modelling features without
fixing one; the reading is the Gaussian image likelihood with a data-based
variance sigma^2 = sigma_bkg^2 + max(d, 0)/t_exp (the noise model of a
background-limited exposure: Gaussian read/background noise plus Poisson
counts over t_exp).  Each pin below fails on a plausible slip: a dropped 1/2,
sigma in place of sigma^2, sigma_bkg unsquared, a missing /t_exp or a missing
max(d, 0).
"""
import math

import numpy as np
from scipy import stats

import oracle as O
import workloads as W


# A 2x2 case worked by hand, with one negative and one zero data pixel.
#   sigma_bkg = 0.1, t_exp = 10
#   d     = [[0.5, -0.2], [1.0, 0.0]]
#   m     = [[0.6,  0.0], [0.8, 0.1]]
#   var   = 0.01 + max(d, 0)/10 = [[0.06, 0.01], [0.11, 0.01]]
#   (m-d)^2 / var = 0.01/0.06 + 0.04/0.01 + 0.04/0.11 + 0.01/0.01
#                 = 1/6 + 4 + 4/11 + 1 = 365/66
#   log L = -365/132
_D = np.array([[0.5, -0.2], [1.0, 0.0]])
_M = np.array([[0.6, 0.0], [0.8, 0.1]])


def test_noise_variance_hand_computed():
    np.testing.assert_allclose(O.noise_variance(_D, 0.1, 10.0), [[0.06, 0.01], [0.11, 0.01]],
                               rtol=1e-14, atol=0)


def test_log_likelihood_hand_computed():
    assert math.isclose(O.log_likelihood(_M, _D, 0.1, 10.0), -365.0 / 132.0, rel_tol=1e-13)


def test_log_likelihood_is_the_gaussian_log_density_up_to_its_normaliser():
    # log L = sum log N(d; m, sigma^2) + 1/2 sum log(2 pi sigma^2): SciPy's normal
    # density fixes both the 1/2 and that sigma^2 (not sigma) divides the residual
    rng = np.random.default_rng(5)
    m = rng.uniform(-0.05, 3.0, (7, 9))
    d = m + rng.normal(0.0, 0.05, m.shape)
    sb, t = 0.03, 250.0
    var = O.noise_variance(d, sb, t)
    expect = float(np.sum(stats.norm.logpdf(d, loc=m, scale=np.sqrt(var)))
                   + 0.5 * np.sum(np.log(2.0 * np.pi * var)))
    assert math.isclose(O.log_likelihood(m, d, sb, t), expect, rel_tol=1e-12)


def test_noise_variance_matches_the_variance_of_the_mock_noise():
    # the seeded mock data d = Poisson(t m)/t + N(0, sigma_bkg^2) has variance
    # m/t + sigma_bkg^2; the data-based reading estimates exactly that, so its
    # mean over many noisy pixels must agree with their sample variance
    sb, t = 0.01, 1000.0
    for level in (0.0, 0.3, 4.0):
        m = np.full((400, 500), level)
        d = W.noisy_image(m, sigma_bkg=sb, t_exp=t, seed=11)
        sample_var = float(d.var())
        expect = sb ** 2 + level / t
        assert abs(sample_var - expect) < 0.01 * expect
        if level > 0.1:     # the data pixels are positive, so max(d, 0) = d on average
            assert abs(float(O.noise_variance(d, sb, t).mean()) - expect) < 0.01 * expect
    # a background-only pixel with negative data takes the background variance alone
    assert O.noise_variance(np.array([-0.5]), sb, t)[0] == sb ** 2


def test_log_likelihood_zero_at_the_data_and_quadratic_in_the_residual():
    rng = np.random.default_rng(6)
    d = rng.uniform(0.0, 2.0, (5, 5))
    assert O.log_likelihood(d, d, 0.01, 1000.0) == 0.0
    e = rng.normal(size=d.shape)
    l1 = O.log_likelihood(d + 1e-3 * e, d, 0.01, 1000.0)
    l2 = O.log_likelihood(d + 2e-3 * e, d, 0.01, 1000.0)
    assert l1 < 0.0 and math.isclose(l2, 4.0 * l1, rel_tol=1e-12)
