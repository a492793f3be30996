"""Image chi^2 log-likelihood (oracle, FP64).

The paper lists several log-likelihood choices among the modelling features and uses autodiff for gradient-based fitting; it fixes neither the
likelihood nor the noise model.  Reading: the Gaussian image likelihood

    log L = -1/2 sum_i (m_i - d_i)^2 / sigma_i^2,
    sigma_i^2 = sigma_bkg^2 + max(d_i, 0) / t_exp,

with the variance taken from the data so that it does not depend on the
model parameters.
"""
import numpy as np


def noise_variance(data, sigma_bkg, t_exp):
    d = np.asarray(data, dtype=np.float64)
    return sigma_bkg ** 2 + np.maximum(d, 0.0) / t_exp


def log_likelihood(model, data, sigma_bkg, t_exp):
    m = np.asarray(model, dtype=np.float64)
    d = np.asarray(data, dtype=np.float64)
    var = noise_variance(d, sigma_bkg, t_exp)
    return -0.5 * float(np.sum((m - d) ** 2 / var))
