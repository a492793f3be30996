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


def convolve_at(img, K, rows, cols):
    """The same convolution evaluated only at the pixels (rows[t], cols[t]),
    each as its own sum over the kernel taps that land inside the image; for
    checking very large images on a sample of outputs."""
    img = np.asarray(img, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    k = K.shape[0]
    c = (k - 1) // 2
    ny, nx = img.shape
    out = np.empty(len(rows), dtype=np.float64)
    for t, (i, j) in enumerate(zip(rows, cols)):
        a0, a1 = max(0, i + c - (ny - 1)), min(k - 1, i + c)
        b0, b1 = max(0, j + c - (nx - 1)), min(k - 1, j + c)
        acc = 0.0
        for a in range(a0, a1 + 1):
            # taps K[a, b0..b1] meet img[i - a + c, j - b + c] for b = b0..b1
            seg = img[i - a + c, j - b1 + c:j - b0 + c + 1][::-1]
            acc += float(np.dot(K[a, b0:b1 + 1], seg))
        out[t] = acc
    return out
