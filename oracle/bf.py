"""Direct bilateral filter, eq. (BF) of Sec. 1, in float64.

    f_BF(i) = sum_{j in Omega} w(j) g(f(i-j) - f(i)) f(i-j)
              / sum_{j in Omega} w(j) g(f(i-j) - f(i)),
    g(t) = exp(-t^2 / (2 sigma_r^2))                       (eq. range_kernel)

Border reading: the paper is silent on what happens where i - j leaves the
image domain I.  Terms with i - j outside I are dropped (the sum runs over
Omega intersected with the shifted domain), which is the same as
zero-extending the auxiliary images of Sec. 3.  Cost O(W^2) per pixel.
"""
from __future__ import annotations

import numpy as np


def range_kernel(t: np.ndarray, sigma_r: float) -> np.ndarray:
    return np.exp(-(t * t) / (2.0 * sigma_r * sigma_r))


def direct_bf(f: np.ndarray, w2: np.ndarray, sigma_r: float) -> np.ndarray:
    """eq. (BF) over the whole image; w2 is the (2W+1)^2 kernel on Omega,
    w2[W + a, W + b] = w((a, b))."""
    f = np.asarray(f, dtype=np.float64)
    H, Wd = f.shape
    W = w2.shape[0] // 2
    num = np.zeros_like(f)
    den = np.zeros_like(f)
    pad = np.zeros((H + 2 * W, Wd + 2 * W))
    valid = np.zeros_like(pad)
    pad[W:W + H, W:W + Wd] = f
    valid[W:W + H, W:W + Wd] = 1.0
    for a in range(-W, W + 1):
        for b in range(-W, W + 1):
            # f(i - j) for j = (a, b): rows r - a, cols c - b
            sh = pad[W - a:W - a + H, W - b:W - b + Wd]
            ok = valid[W - a:W - a + H, W - b:W - b + Wd]
            k = w2[W + a, W + b] * range_kernel(sh - f, sigma_r) * ok
            num += k * sh
            den += k
    return num / den


def direct_bf_at(f: np.ndarray, pixels: np.ndarray, w2: np.ndarray,
                 sigma_r: float) -> np.ndarray:
    """eq. (BF) at the listed pixels only ((M, 2) array of (row, col))."""
    f = np.asarray(f, dtype=np.float64)
    H, Wd = f.shape
    W = w2.shape[0] // 2
    out = np.empty(len(pixels))
    for m, (r, c) in enumerate(pixels):
        r0, r1 = max(0, r - W), min(H, r + W + 1)
        c0, c1 = max(0, c - W), min(Wd, c + W + 1)
        win = f[r0:r1, c0:c1]
        # pixel (rr, cc) = i - j  ->  j = (r - rr, c - cc)
        wj = w2[W + r - np.arange(r0, r1)][:, W + c - np.arange(c0, c1)]
        k = wj * range_kernel(win - f[r, c], sigma_r)
        out[m] = (k * win).sum() / k.sum()
    return out
