"""Spatial kernels of the bilateral filter (Sec. 1, eqs. spatial_kernel1 and
spatial_kernel2).

The support is the square Omega = [-W, W] x [-W, W]; for the Gaussian kernel
the paper sets W = 3 sigma_s, read here as W = ceil(3 sigma_s) so that W is
an integer for any sigma_s.  Both kernels are separable, w(a, b) =
w1(a) w1(b), and are returned as the 1-D factor w1 over a = -W..W.

Normalisation does not change eq. (BF) or eq. (GPA) (w appears in the
numerator and the denominator).  It matters only for w(0) in Prop.
(accuracy) and Cor. (eps), where the paper assumes sum_Omega w = 1; w0()
returns that normalised centre weight.
"""
from __future__ import annotations

import math

import numpy as np

BOX = "box"
GAUSS = "gauss"


def support(kind: str, sigma_s: float | None = None, W: int | None = None) -> int:
    """Half-width W of Omega.  Box: W given.  Gaussian: W given, else ceil(3 sigma_s)."""
    if W is not None:
        return int(W)
    if kind != GAUSS or sigma_s is None:
        raise ValueError("W is required for the box kernel")
    return int(math.ceil(3.0 * sigma_s - 1e-12))


def taps1d(kind: str, sigma_s: float | None = None, W: int | None = None) -> np.ndarray:
    """1-D factor w1(a), a = -W..W, unnormalised (box: all ones; Gaussian:
    exp(-a^2 / (2 sigma_s^2)), eq. spatial_kernel1 restricted to one axis)."""
    W = support(kind, sigma_s, W)
    a = np.arange(-W, W + 1, dtype=np.float64)
    if kind == BOX:
        return np.ones_like(a)
    if kind == GAUSS:
        return np.exp(-(a * a) / (2.0 * sigma_s * sigma_s))
    raise ValueError(kind)


def taps2d(kind: str, sigma_s: float | None = None, W: int | None = None) -> np.ndarray:
    """Full (2W+1)^2 kernel w(a, b) on Omega (unnormalised)."""
    t = taps1d(kind, sigma_s, W)
    return np.outer(t, t)


def w0(kind: str, sigma_s: float | None = None, W: int | None = None) -> float:
    """w(0) of the kernel normalised to sum 1 over Omega (Prop. accuracy)."""
    w = taps2d(kind, sigma_s, W)
    c = w.shape[0] // 2
    return float(w[c, c] / w.sum())
