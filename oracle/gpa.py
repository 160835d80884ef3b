"""Gaussian-Polynomial Approximation of the bilateral filter (Sec. 2-3), in
float64.

Two independent evaluations of the same filter are given:

* ``gpa_pairwise`` evaluates eq. (GPA) directly: eq. (BF) with the range
  kernel replaced by the Gaussian-polynomial of eq. (GaussPolynomial),
  pair by pair, O(W^2 N) per pixel.  The arguments of phi_N are
  (t, tau) = (h(i-j), h(i)) on the centred image h = f - c (Sec. 2:
  t = f(i-j), tau = f(i); Sec. 3, eq. shift: the intensities are centred
  before the expansion, and the centre is added back at the end).
* ``gpa_alg2`` evaluates the form Algorithm 2 (Sec. 3) computes: the N+1
  auxiliary images F_n = exp(-h^2/2 sigma_r^2) (h/sigma_r)^n of
  eq. (intImg), each filtered with the spatial kernel (eq.
  spatialFiltering), and the numerator P and denominator Q of eqs. (P),
  (Q) summed over n with the weights G_n/n! (``gpa_sums``; the other
  modules pass their own spatial filter to it).

Appendix B shows the two agree in exact arithmetic; the tests pin that.
"Order N" is the number of Taylor terms n = 0..N-1 of eq. (approx), so
Algorithm 2 performs N+1 spatial filterings (of F_0..F_N).

Border: zero extension of the auxiliary images (equivalently, Omega is
truncated to the image in eq. BF / eq. GPA), as in ``oracle.bf``.

Small sigma_r: the partial sums of ``phi`` reach e^{|s|} with |s| up to
lambda = T^2 / sigma_r^2 and overflow float64 beyond lambda ~ 709 (sigma_r
below about 4.8 on [0, 255]).  ``phi_wide`` evaluates the same sum with
every term formed in log space, which stays finite to lambda = 1400; the
pair-by-pair forms take it with ``wide=True``.

Test infrastructure only: the product path never imports this package.
"""
from __future__ import annotations

import math

import numpy as np


def phi(t: np.ndarray, tau: np.ndarray, sigma_r: float, N: int) -> np.ndarray:
    """Gaussian-polynomial phi_{N, sigma_r}(t, tau), eq. (GaussPolynomial):
    exp(-(t^2 + tau^2) / (2 sigma_r^2)) * sum_{n=0}^{N-1} (tau t / sigma_r^2)^n / n!"""
    t = np.asarray(t, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    s = tau * t / (sigma_r * sigma_r)
    term = np.ones(np.broadcast(t, tau).shape)
    acc = np.zeros_like(term)
    for n in range(N):
        if n > 0:
            term = term * s / n
        acc = acc + term
    return np.exp(-(t * t + tau * tau) / (2.0 * sigma_r * sigma_r)) * acc


def phi_wide(t: np.ndarray, tau: np.ndarray, sigma_r: float, N: int) -> np.ndarray:
    """phi_{N, sigma_r}(t, tau) of eq. (GaussPolynomial), each term
    exp(-(t^2 + tau^2) / (2 sigma_r^2)) s^n / n!, s = tau t / sigma_r^2,
    taken as sign(s)^n exp(-(t^2 + tau^2) / (2 sigma_r^2) + n log|s| - log n!):
    every term is at most exp(-(|t| - |tau|)^2 / (2 sigma_r^2)) <= 1."""
    t = np.asarray(t, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    s = tau * t / (sigma_r * sigma_r)
    base = -(t * t + tau * tau) / (2.0 * sigma_r * sigma_r)
    with np.errstate(divide="ignore"):
        ls = np.log(np.abs(s))
    neg = s < 0
    acc = np.zeros(np.broadcast(t, tau).shape)
    for n in range(N):
        if n == 0:
            term = np.exp(base) * np.ones_like(acc)
        else:
            term = np.exp(base + n * ls - math.lgamma(n + 1.0))
            if n % 2 == 1:
                term = np.where(neg, -term, term)
        acc = acc + term
    return acc


def kernel_error(t, tau, sigma_r: float, N: int) -> np.ndarray:
    """E_{N, sigma_r}(t, tau) = g(t - tau) - phi_N(t, tau), eq. (error)."""
    t = np.asarray(t, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    g = np.exp(-((t - tau) ** 2) / (2.0 * sigma_r * sigma_r))
    return g - phi(t, tau, sigma_r, N)


def gpa_pairwise(f: np.ndarray, w2: np.ndarray, sigma_r: float, N: int,
                 center: float, wide: bool = False) -> np.ndarray:
    """eq. (GPA) on the centred image h = f - center, plus center (Prop. centering).
    wide: phi evaluated by ``phi_wide``."""
    ph = phi_wide if wide else phi
    h = np.asarray(f, dtype=np.float64) - center
    H, Wd = h.shape
    W = w2.shape[0] // 2
    num = np.zeros_like(h)
    den = np.zeros_like(h)
    pad = np.zeros((H + 2 * W, Wd + 2 * W))
    valid = np.zeros_like(pad)
    pad[W:W + H, W:W + Wd] = h
    valid[W:W + H, W:W + Wd] = 1.0
    for a in range(-W, W + 1):
        for b in range(-W, W + 1):
            sh = pad[W - a:W - a + H, W - b:W - b + Wd]
            ok = valid[W - a:W - a + H, W - b:W - b + Wd]
            k = w2[W + a, W + b] * ph(sh, h, sigma_r, N) * ok
            num += k * sh
            den += k
    return num / den + center


def gpa_pairwise_at(f: np.ndarray, pixels: np.ndarray, w2: np.ndarray,
                    sigma_r: float, N: int, center: float, wide: bool = False) -> np.ndarray:
    """eq. (GPA) at the listed (row, col) pixels only (wide: ``phi_wide``)."""
    ph = phi_wide if wide else phi
    h = np.asarray(f, dtype=np.float64) - center
    H, Wd = h.shape
    W = w2.shape[0] // 2
    out = np.empty(len(pixels))
    for m, (r, c) in enumerate(pixels):
        r0, r1 = max(0, r - W), min(H, r + W + 1)
        c0, c1 = max(0, c - W), min(Wd, c + W + 1)
        win = h[r0:r1, c0:c1]
        wj = w2[W + r - np.arange(r0, r1)][:, W + c - np.arange(c0, c1)]
        k = wj * ph(win, h[r, c], sigma_r, N)
        out[m] = (k * win).sum() / k.sum() + center
    return out


def spatial_filter(F: np.ndarray, w1: np.ndarray) -> np.ndarray:
    """F_bar(i) = sum_{j in Omega} w(j) F(i - j), eq. (spatialFiltering), for
    the separable kernel w(a, b) = w1(a) w1(b), with F zero outside the image."""
    F = np.asarray(F, dtype=np.float64)
    W = len(w1) // 2
    H, Wd = F.shape
    tmp = np.zeros_like(F)
    for a in range(-W, W + 1):          # rows: tmp(r, c) = sum_a w1(a) F(r - a, c)
        lo, hi = max(0, a), min(H, H + a)
        if hi > lo:
            tmp[lo:hi, :] += w1[W + a] * F[lo - a:hi - a, :]
    out = np.zeros_like(F)
    for b in range(-W, W + 1):          # cols: out(r, c) = sum_b w1(b) tmp(r, c - b)
        lo, hi = max(0, b), min(Wd, Wd + b)
        if hi > lo:
            out[:, lo:hi] += w1[W + b] * tmp[:, lo - b:hi - b]
    return out


def power_over_factorial(u: np.ndarray, N: int):
    """The weights u^n / n! of eqs. (P) and (Q) for n = 0 .. N-1 (G_n(i)/n!
    with G_n = u^n of eq. intImg), each the product of the n factors u/k,
    k = 1 .. n, so that no power or factorial leaves the float64 range."""
    c = np.ones_like(u)
    for n in range(N):
        yield n, c
        c = c * (u / (n + 1))


def gpa_sums(f: np.ndarray, filt, sigma_r: float, N: int, T: float):
    """Eqs. (intImg), (spatialFiltering), (P), (Q) and (PbyQ) of Sec. 3 for
    the image centred by eq. (shift) with t_c = T, h = f - T, u = h/sigma_r:

        F_n = exp(-u^2/2) u^n,   Fbar_n = filt(F_n)            n = 0 .. N
        Q   = sum_{n<N} u^n/n! Fbar_n
        P   = sigma_r sum_{n<N} u^n/n! Fbar_{n+1}
        out = P / Q + T

    `filt` is the spatial filtering of eq. (spatialFiltering) (any border
    rule and any number of axes).  Every F_n is formed from its definition and
    filtered once, N + 1 filterings in all.  Returns (out, P, Q)."""
    f = np.asarray(f, dtype=np.float64)
    u = (f - T) / sigma_r
    E = np.exp(-0.5 * u * u)
    P = np.zeros_like(f)
    Q = np.zeros_like(f)
    Fbar_n = filt(E)
    un = np.ones_like(u)   # u^(n+1) below, one factor u per order
    for n, c in power_over_factorial(u, N):
        un = un * u
        Fbar_next = filt(E * un)
        Q += c * Fbar_n
        P += c * Fbar_next
        Fbar_n = Fbar_next
    P *= sigma_r
    return P / Q + T, P, Q


def gpa_alg2(f: np.ndarray, w1: np.ndarray, sigma_r: float, N: int, T: float,
             return_pq: bool = False):
    """The N + 1 filtering form of eq. (GPA) (eqs. P, Q, PbyQ; Algorithm 2
    computes the same sums) with the separable zero-extension filter
    ``spatial_filter``.  T is the centre of the dynamic range [0, 2T] (the
    paper centres with t_c = T).  return_pq: also P and Q."""
    out, P, Q = gpa_sums(f, lambda F: spatial_filter(F, w1), sigma_r, N, T)
    if return_pq:
        return out, P, Q
    return out
