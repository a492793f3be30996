"""Linear amplitude solver (oracle, FP64).  Test infrastructure only.

The paper lists lenstronomy's linear amplitude solver among the features it
keeps (section "Why JAXtronomy?"): the simulated image is linear in each light
component's amplitude, so the amplitudes need not be sampled.  Definition
(reading): with the basis images

    B_j = PSF * (image of light component j alone at unit amplitude),

components ordered as the source list, then the lens-light list, the
amplitudes minimise the weighted squared residual

    a = argmin_a  sum_i w_i (d_i - sum_j a_j B_j,i)^2,

the model is sum_j a_j B_j and log L = -1/2 sum_i w_i (d_i - m_i)^2.  The
weighted least-squares problem is solved by a library routine (NumPy's lstsq
on the rows scaled by sqrt(w)).
"""
import copy

import numpy as np

from .simulate import simulate_image


def basis_images(scene):
    """(n, ny, nx): the image of each component alone at unit amplitude,
    sources first, then lens light."""
    out = []
    comps = [("source", i) for i in range(len(scene.source))] + \
            [("lens_light", i) for i in range(len(scene.lens_light))]
    for which, i in comps:
        sc = copy.copy(scene)
        c = copy.copy(getattr(scene, which)[i])
        c.amp = 1.0
        sc.source = [c] if which == "source" else []
        sc.lens_light = [c] if which == "lens_light" else []
        out.append(simulate_image(sc))
    return np.array(out)


def linear_amplitudes(scene, data, inv_var, basis=None):
    """Amplitudes, model image and log-likelihood of the weighted linear fit."""
    B = basis_images(scene) if basis is None else np.asarray(basis, dtype=np.float64)
    n = B.shape[0]
    d = np.asarray(data, dtype=np.float64).reshape(-1)
    w = np.asarray(inv_var, dtype=np.float64).reshape(-1)
    A = B.reshape(n, -1).T
    sw = np.sqrt(w)
    amps, *_ = np.linalg.lstsq(A * sw[:, None], d * sw, rcond=None)
    model = (A @ amps).reshape(B.shape[1:])
    logL = -0.5 * float(np.sum(w * (d - model.reshape(-1)) ** 2))
    return amps, model, logL
