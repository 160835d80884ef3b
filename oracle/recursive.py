"""Recursive (Deriche) Gaussian spatial kernel, and the bilateral filter and
its Gaussian-polynomial approximation with it, in float64.  Test
infrastructure only.

Sec. 1 and Sec. 3 (after eqs. (P), (Q)) note that the N+1 spatial
filterings of eq. (spatialFiltering) cost O(1) per pixel for a Gaussian w
when w is implemented recursively, citing Deriche's 1993 report.  Deriche
fits the sampled Gaussian exp(-x^2/2), x = n/sigma_s, with two damped
oscillations,

    h(n) = (a0 cos(w0 x) + a1 sin(w0 x)) e^{-b0 x}
         + (c0 cos(w1 x) + c1 sin(w1 x)) e^{-b1 x},    x = |n| / sigma_s,

a0 = 1.680, a1 = 3.735, b0 = 1.783, w0 = 0.6318, c0 = -0.6803, c1 = -0.2598,
b1 = 1.723, w1 = 1.997 (the fit of his report; h(0) = 0.9997).  Because h on
n >= 0 is a sum of geometric sequences, convolving with h(|n|) splits into a
causal part (n >= 0) and an anticausal part (n >= 1), each a short linear
recursion: the filter costs O(1) per sample whatever sigma_s.

What the recursions compute has a plain definition, and that is what this
module uses: the 2-D kernel w(a, b) = h(|a|) h(|b|) of unbounded support,
applied to the zero-extended image (the border reading of ``oracle.bf``), is
``spatial_filter`` = K_H F K_W^T with the Toeplitz matrices K_L[i, j] =
h(|i - j|).  ``iir_filter_lines`` is the recursive evaluation, written here
only so the tests can pin that the recursions reproduce the definition (it is
not used by the filters below).

The fit has small negative lobes (min h = -1.4e-4 near x = 5.4), so the
spatial weights are not all positive; the normalised centre weight used by
the order rule is w(0) = (h(0) / sum_n h(|n|))^2.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from . import bf as _bf
from . import gpa as _gpa

# Deriche's fit of the Gaussian: (a, a', b, omega) of the two damped oscillations
FIT = ((1.680, 3.735, 1.783, 0.6318), (-0.6803, -0.2598, 1.723, 1.997))


def kernel(n: np.ndarray, sigma_s: float) -> np.ndarray:
    """h(|n|), the closed form above."""
    x = np.abs(np.asarray(n, dtype=np.float64)) / sigma_s
    out = np.zeros_like(x)
    for a, ap, b, om in FIT:
        out += (a * np.cos(om * x) + ap * np.sin(om * x)) * np.exp(-b * x)
    return out


def kernel_sum(sigma_s: float) -> float:
    """sum over all integers n of h(|n|), by direct summation until the terms vanish."""
    n = np.arange(1, int(60 * sigma_s) + 64)
    return float(kernel(0, sigma_s) + 2.0 * kernel(n, sigma_s).sum())


def w0(sigma_s: float) -> float:
    """Normalised centre weight of the 2-D kernel h(|a|) h(|b|)."""
    return (float(kernel(0, sigma_s)) / kernel_sum(sigma_s)) ** 2


@lru_cache(maxsize=8)
def _toeplitz(L: int, sigma_s: float) -> np.ndarray:
    i = np.arange(L)
    K = kernel(i[:, None] - i[None, :], sigma_s)
    K.setflags(write=False)
    return K


def toeplitz(L: int, sigma_s: float) -> np.ndarray:
    """K[i, j] = h(|i - j|) for a line of L samples (cached, read-only)."""
    return _toeplitz(int(L), float(sigma_s))


def spatial_filter(F: np.ndarray, sigma_s: float) -> np.ndarray:
    """eq. (spatialFiltering) with w(a, b) = h(|a|) h(|b|) over the whole
    zero-extended image: F_bar = K_H F K_W^T."""
    F = np.asarray(F, dtype=np.float64)
    H, Wd = F.shape
    return toeplitz(H, sigma_s) @ F @ toeplitz(Wd, sigma_s).T


def kernel2d(sigma_s: float, half: int) -> np.ndarray:
    """w(a, b) = h(|a|) h(|b|) for |a|, |b| <= half (covers an image of side half + 1)."""
    h = kernel(np.arange(-half, half + 1), sigma_s)
    return np.outer(h, h)


def direct_bf(f: np.ndarray, sigma_s: float, sigma_r: float) -> np.ndarray:
    """eq. (BF) with the recursive-Gaussian spatial kernel (unbounded support)."""
    H, Wd = np.shape(f)
    return _bf.direct_bf(f, kernel2d(sigma_s, max(H, Wd) - 1), sigma_r)


def gpa_pairwise(f: np.ndarray, sigma_s: float, sigma_r: float, N: int, center: float) -> np.ndarray:
    """eq. (GPA) pair by pair with the recursive-Gaussian spatial kernel."""
    H, Wd = np.shape(f)
    return _gpa.gpa_pairwise(f, kernel2d(sigma_s, max(H, Wd) - 1), sigma_r, N, center)


def gpa_alg2(f: np.ndarray, sigma_s: float, sigma_r: float, N: int, T: float) -> np.ndarray:
    """Eqs. (P), (Q), (PbyQ) (the sums of ``oracle.gpa.gpa_sums``) with
    ``spatial_filter`` above as eq. (spatialFiltering): N+1 filterings."""
    return _gpa.gpa_sums(f, lambda F: spatial_filter(F, sigma_s), sigma_r, N, T)[0]


def gpa_alg2_at(f: np.ndarray, pixels: np.ndarray, sigma_s: float, sigma_r: float, N: int,
                T: float) -> np.ndarray:
    """``gpa_alg2`` at the listed (row, col) pixels only: F_bar_n there is
    k_r^T F_n k_c with the rows k_r = h(|r - i|), k_c = h(|c - j|)."""
    f = np.asarray(f, dtype=np.float64)
    H, Wd = f.shape
    px = np.asarray(pixels)
    rr, cc = px[:, 0], px[:, 1]
    Kr = kernel(rr[:, None] - np.arange(H)[None, :], sigma_s)
    Kc = kernel(cc[:, None] - np.arange(Wd)[None, :], sigma_s)
    u = (f - T) / sigma_r
    E = np.exp(-0.5 * u * u)

    def at(F):
        return ((Kr @ F) * Kc).sum(axis=1)

    P = np.zeros(len(px))
    Q = np.zeros(len(px))
    Fbar_n = at(E)
    un = np.ones_like(u)   # u^(n+1) below, one factor u per order
    for n, c in _gpa.power_over_factorial(u[rr, cc], N):
        un = un * u
        Fbar_next = at(E * un)
        Q += c * Fbar_n
        P += c * Fbar_next
        Fbar_n = Fbar_next
    return sigma_r * P / Q + T


def iir_sections(sigma_s: float):
    """Per damped oscillation (a, a', b, omega), with rho = e^{-b/sigma_s} and
    theta = omega/sigma_s, the causal and anticausal recursions whose impulse
    responses are h_j(n), n >= 0, and h_j(m), m >= 1:

        u[i] = a x[i] + (a' rho sin - a rho cos) x[i-1] + 2 rho cos u[i-1] - rho^2 u[i-2]
        v[i] = (a' rho sin + a rho cos) x[i+1] - a rho^2 x[i+2] + 2 rho cos v[i+1] - rho^2 v[i+2]

    (the z-transforms of rho^n cos(n theta) and rho^n sin(n theta)).  Returns
    a list of (b0, b1, c0, c1, p1, p2): u uses (b0, b1), v uses (c0, c1), both
    use the feedback p1 = 2 rho cos theta, p2 = -rho^2."""
    out = []
    for a, ap, b, om in FIT:
        rho, th = np.exp(-b / sigma_s), om / sigma_s
        cs, sn = rho * np.cos(th), rho * np.sin(th)
        out.append((a, ap * sn - a * cs, ap * sn + a * cs, -a * rho * rho, 2.0 * cs, -rho * rho))
    return out


def iir_filter_lines(X: np.ndarray, sigma_s: float) -> np.ndarray:
    """The recursive evaluation of sum_j h(|i - j|) x[j] along axis 1 of X
    (each row a zero-extended line): causal plus anticausal recursions of
    both oscillations, run with zero state from the line ends."""
    X = np.asarray(X, dtype=np.float64)
    L = X.shape[1]
    Y = np.zeros_like(X)
    for b0, b1, c0, c1, p1, p2 in iir_sections(sigma_s):
        u1 = np.zeros(X.shape[0])
        u2 = np.zeros(X.shape[0])
        xm = np.zeros(X.shape[0])
        for i in range(L):
            u = b0 * X[:, i] + b1 * xm + p1 * u1 + p2 * u2
            Y[:, i] += u
            u2, u1, xm = u1, u, X[:, i]
        v1 = np.zeros(X.shape[0])
        v2 = np.zeros(X.shape[0])
        x1 = np.zeros(X.shape[0])
        x2 = np.zeros(X.shape[0])
        for i in range(L - 1, -1, -1):
            v = c0 * x1 + c1 * x2 + p1 * v1 + p2 * v2
            Y[:, i] += v
            v2, v1 = v1, v
            x2, x1 = x1, X[:, i]
    return Y
