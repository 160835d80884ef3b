"""Approximation order N and the error bounds of Sec. 2-3, in float64.

* poisson_tail(N, lam)   Prop. (upperBound): ||E_N||_inf <= sum_{n>=N}
                         e^{-lam} lam^n / n!,  lam = T^2 / sigma_r^2; the
                         right side is Prob(X >= N) for X ~ Poisson(lam),
                         i.e. the regularised lower incomplete gamma P(N, lam).
* chernoff_order         Prop. (LambW): the smallest integer N > lam with
                         e^{-lam} (e lam)^N / N^N <= eps (eq. inequality) is
                         ceil(q / W0(q e^{-p})), p = 1 + log lam,
                         q = -lam - log eps (W0: principal Lambert-W branch).
* chernoff_order_bisect  the same root theta > lam of
                         nu(x) = x log x - p x - q (App. A), by bisection.
* alg1_order             Algorithm 1 as printed (sigma_r >= 70 -> 10; else
                         the 4-term series of eq. (series) and, for
                         sigma_r < 30, three Newton steps, eq. Newton_method).
* eps_from_delta         Cor. (eps): eps = w(0) delta / (2T + delta).
* accuracy_bound         Prop. (accuracy): 2 T ||E|| / (w(0) - ||E||).
* nvsdelta               eq. (Nvsdelta), the asymptotic order of App. D.
* kernel_error_max_grid  max |E_N(t, tau)| over a grid of [-T, T]^2 (eq. Linf).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import gammainc, lambertw


def lam_of(T: float, sigma_r: float) -> float:
    return (T / sigma_r) ** 2


def poisson_tail(N: int, lam: float) -> float:
    """sum_{n >= N} e^{-lam} lam^n / n!  (Prop. upperBound)."""
    if N <= 0:
        return 1.0
    return float(gammainc(N, lam))


def _pq(lam: float, eps: float):
    p = 1.0 + math.log(lam)
    q = -lam - math.log(eps)
    return p, q


def chernoff_theta(lam: float, eps: float) -> float:
    """theta = q / W0(q e^{-p}) (Prop. LambW), the real root > lam of nu."""
    p, q = _pq(lam, eps)
    w = lambertw(q * math.exp(-p), 0)
    return float(q / w.real)


def chernoff_order(lam: float, eps: float) -> int:
    """N0 = ceil(q / W0(q e^{-p})), eq. (LambW); '[x]' is the ceiling (Sec. 2)."""
    return int(math.ceil(chernoff_theta(lam, eps) - 1e-12))


def chernoff_order_bisect(lam: float, eps: float) -> int:
    """Smallest integer x > lam with nu(x) = x log x - p x - q >= 0 (App. A),
    located by bisection on the convex nu (minimum at x = lam)."""
    p, q = _pq(lam, eps)

    def nu(x):
        return x * math.log(x) - p * x - q

    lo = lam
    hi = max(2.0 * lam, lam + 1.0)
    while nu(hi) < 0.0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if nu(mid) < 0.0:
            lo = mid
        else:
            hi = mid
    return int(math.ceil(hi - 1e-12))


def series_w0(t: float) -> float:
    """First four terms of the Lambert-W series, eq. (series):
    W0(t) ~ t - t^2 + 3 t^3 / 2 - 8 t^4 / 3."""
    return t - t * t + 1.5 * t ** 3 - (8.0 / 3.0) * t ** 4


def newton_step(x: float, p: float, q: float) -> float:
    """One Newton step on nu(x) = x log x - p x - q, eq. (Newton_method)."""
    return x - (x * math.log(x) - p * x - q) / (math.log(x) + 1.0 - p)


def series_order(lam: float, eps: float, newton_steps: int = 0) -> int:
    """ceil(q / W0_series(q / (e lam))) optionally refined by Newton steps
    (the N''_0 and N'''_0 rows of Table 1)."""
    p, q = _pq(lam, eps)
    t = q / (math.e * lam)
    x = q / series_w0(t)
    for _ in range(newton_steps):
        x = newton_step(x, p, q)
    return int(math.ceil(x - 1e-12))


def alg1_order(sigma_r: float, eps: float, T: float) -> int:
    """Algorithm 1 as printed, with the series term -8t^4/3 of eq. (series)."""
    if sigma_r >= 70.0:
        return 10
    lam = lam_of(T, sigma_r)
    return series_order(lam, eps, newton_steps=3 if sigma_r < 30.0 else 0)


def poisson_order(lam: float, eps: float) -> int:
    """Smallest N >= 1 whose Poisson tail (Prop. upperBound) is <= eps."""
    N = 1
    while poisson_tail(N, lam) > eps:
        N += 1
    return N


def eps_from_delta(delta: float, w0: float, T: float) -> float:
    """Cor. (eps): kernel tolerance that guarantees +-delta filtering accuracy."""
    return w0 * delta / (2.0 * T + delta)


def accuracy_bound(E: float, w0: float, T: float) -> float:
    """Prop. (accuracy): ||f_BF - f_GPA||_inf <= 2 T ||E|| / (w(0) - ||E||)."""
    if E >= w0:
        return math.inf
    return 2.0 * T * E / (w0 - E)


def nvsdelta(T: float, sigma_r: float, w0: float, delta: float) -> float:
    """eq. (Nvsdelta): N0 ~ 1.72 (T / sigma_r)^2 + log(2T / (w(0) delta))."""
    return 1.72 * (T / sigma_r) ** 2 + math.log(2.0 * T / (w0 * delta))


def order_for_delta(delta: float, w0: float, T: float, sigma_r: float) -> int:
    """The default planning rule: eps from Cor. (eps), N from Prop. (LambW)."""
    return chernoff_order(lam_of(T, sigma_r), eps_from_delta(delta, w0, T))


def kernel_error_max_grid(N: int, sigma_r: float, T: float, n: int = 257) -> float:
    """max |E_N(t, tau)| over an n x n grid of [-T, T]^2 (eq. Linf)."""
    from .gpa import kernel_error
    g = np.linspace(-T, T, n)
    t, tau = np.meshgrid(g, g, indexing="ij")
    return float(np.abs(kernel_error(t, tau, sigma_r, N)).max())
