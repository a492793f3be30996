"""PSF convolution (oracle, FP64).

The paper's third step convolves the lensed image with the PSF
(image-simulation section; its FFT-convolution section times the same
operation through an FFT).  Reading of the unstated conventions: a true
convolution (the kernel is flipped), odd kernel size k, zero padding outside
the image, output of the input's size ("same"):

    out[i, j] = sum_{a, b} K[a, b] * img[i - a + c, j - b + c],  c = (k-1)/2.

The definition is evaluated literally, one kernel tap at a time.
"""
import numpy as np


def convolve_same(img, K):
    img = np.asarray(img, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    k = K.shape[0]
    if K.shape != (k, k) or k % 2 != 1:
        raise ValueError("kernel must be square with odd size")
    c = (k - 1) // 2
    ny, nx = img.shape
    pad = np.zeros((ny + 2 * c, nx + 2 * c), dtype=np.float64)
    pad[c:c + ny, c:c + nx] = img
    out = np.zeros_like(img)
    # img[i - a + c, j - b + c] == pad[i - a + 2c, j - b + 2c]
    for a in range(k):
        for b in range(k):
            w = K[a, b]
            if w != 0.0:
                out += w * pad[2 * c - a:2 * c - a + ny, 2 * c - b:2 * c - b + nx]
    return out
