"""Cross (joint) bilateral filter and its Gaussian-polynomial approximation,
in float64.  Test infrastructure only.

Sec. 1 (Introduction) and Sec. 5 (Conclusion) name the cross (joint)
bilateral filter as a direct extension of the method: the range kernel is
evaluated on a guide image h while the averaged values come from f,

    f_CBF(i) = sum_{j in Omega} w(j) g(h(i-j) - h(i)) f(i-j)
               / sum_{j in Omega} w(j) g(h(i-j) - h(i)),

with g of eq. (range_kernel).  Replacing g by phi_N (eq. GaussPolynomial)
on the centred guide (eq. shift) and expanding as in Sec. 3 gives, with
x = (h - c)/sigma_r, F_n = exp(-x^2/2) x^n (eq. intImg on the guide) and
G_n = F_n at the centre pixel,

    Q(i) = sum_{n<N} G_n(i)/n! (w * F_n)(i),
    P(i) = sum_{n<N} G_n(i)/n! (w * (F_n f))(i),      out = P / Q,

i.e. 2N spatial filterings.  With h = f the numerator is f = c + sigma_r x,
which turns (w * (F_n f)) into c (w * F_n) + sigma_r (w * F_{n+1}) and gives
back eqs. (P), (Q), (PbyQ) of the plain filter; the tests pin that identity.

Border: zero extension of the auxiliary images, as in ``oracle.bf``.
"""
from __future__ import annotations

import numpy as np

from .bf import range_kernel
from .gpa import phi, power_over_factorial, spatial_filter


def direct_joint_bf(f: np.ndarray, h: np.ndarray, w2: np.ndarray, sigma_r: float) -> np.ndarray:
    """The cross bilateral filter as written above, over the whole image."""
    f = np.asarray(f, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    H, Wd = f.shape
    W = w2.shape[0] // 2
    num = np.zeros_like(f)
    den = np.zeros_like(f)
    padf = np.zeros((H + 2 * W, Wd + 2 * W))
    padh = np.zeros_like(padf)
    valid = np.zeros_like(padf)
    padf[W:W + H, W:W + Wd] = f
    padh[W:W + H, W:W + Wd] = h
    valid[W:W + H, W:W + Wd] = 1.0
    for a in range(-W, W + 1):
        for b in range(-W, W + 1):
            sf = padf[W - a:W - a + H, W - b:W - b + Wd]
            sh = padh[W - a:W - a + H, W - b:W - b + Wd]
            ok = valid[W - a:W - a + H, W - b:W - b + Wd]
            k = w2[W + a, W + b] * range_kernel(sh - h, sigma_r) * ok
            num += k * sf
            den += k
    return num / den


def direct_joint_bf_at(f: np.ndarray, h: np.ndarray, pixels: np.ndarray, w2: np.ndarray,
                       sigma_r: float) -> np.ndarray:
    """The cross bilateral filter at the listed (row, col) pixels only."""
    f = np.asarray(f, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    H, Wd = f.shape
    W = w2.shape[0] // 2
    out = np.empty(len(pixels))
    for m, (r, c) in enumerate(pixels):
        r0, r1 = max(0, r - W), min(H, r + W + 1)
        c0, c1 = max(0, c - W), min(Wd, c + W + 1)
        wj = w2[W + r - np.arange(r0, r1)][:, W + c - np.arange(c0, c1)]
        k = wj * range_kernel(h[r0:r1, c0:c1] - h[r, c], sigma_r)
        out[m] = (k * f[r0:r1, c0:c1]).sum() / k.sum()
    return out


def gpa_joint_pairwise(f: np.ndarray, h: np.ndarray, w2: np.ndarray, sigma_r: float, N: int,
                       center: float) -> np.ndarray:
    """The cross filter with g replaced by phi_N on the centred guide, pair by pair."""
    f = np.asarray(f, dtype=np.float64)
    hc = np.asarray(h, dtype=np.float64) - center
    H, Wd = f.shape
    W = w2.shape[0] // 2
    num = np.zeros_like(f)
    den = np.zeros_like(f)
    padf = np.zeros((H + 2 * W, Wd + 2 * W))
    padh = np.zeros_like(padf)
    valid = np.zeros_like(padf)
    padf[W:W + H, W:W + Wd] = f
    padh[W:W + H, W:W + Wd] = hc
    valid[W:W + H, W:W + Wd] = 1.0
    for a in range(-W, W + 1):
        for b in range(-W, W + 1):
            sf = padf[W - a:W - a + H, W - b:W - b + Wd]
            sh = padh[W - a:W - a + H, W - b:W - b + Wd]
            ok = valid[W - a:W - a + H, W - b:W - b + Wd]
            k = w2[W + a, W + b] * phi(sh, hc, sigma_r, N) * ok
            num += k * sf
            den += k
    return num / den


def gpa_joint_pairwise_at(f: np.ndarray, h: np.ndarray, pixels: np.ndarray, w2: np.ndarray,
                          sigma_r: float, N: int, center: float) -> np.ndarray:
    """gpa_joint_pairwise at the listed (row, col) pixels only."""
    f = np.asarray(f, dtype=np.float64)
    hc = np.asarray(h, dtype=np.float64) - center
    H, Wd = f.shape
    W = w2.shape[0] // 2
    out = np.empty(len(pixels))
    for m, (r, c) in enumerate(pixels):
        r0, r1 = max(0, r - W), min(H, r + W + 1)
        c0, c1 = max(0, c - W), min(Wd, c + W + 1)
        wj = w2[W + r - np.arange(r0, r1)][:, W + c - np.arange(c0, c1)]
        k = wj * phi(hc[r0:r1, c0:c1], hc[r, c], sigma_r, N)
        out[m] = (k * f[r0:r1, c0:c1]).sum() / k.sum()
    return out


def gpa_joint_alg2(f: np.ndarray, h: np.ndarray, w1: np.ndarray, sigma_r: float, N: int,
                   T: float) -> np.ndarray:
    """The filtering form of the cross filter written above: F_n = exp(-x^2/2)
    x^n of the centred guide (eq. intImg), 2N spatial filterings (of F_n and of
    F_n f), weights x^n/n! at the centre pixel, out = P / Q."""
    f = np.asarray(f, dtype=np.float64)
    x = (np.asarray(h, dtype=np.float64) - T) / sigma_r
    E = np.exp(-0.5 * x * x)
    P = np.zeros_like(f)
    Q = np.zeros_like(f)
    xn = np.ones_like(x)   # x^n, one factor x per order
    for n, c in power_over_factorial(x, N):
        Fn = E * xn
        Q += c * spatial_filter(Fn, w1)
        P += c * spatial_filter(Fn * f, w1)
        xn = xn * x
    return P / Q
