"""The bilateral filter and its Gaussian-polynomial approximation on video
and volume data, in float64.  Test infrastructure only.

Sec. 1 and Sec. 5 note that the filter extends directly to video and volume
data: the domain becomes I in Z^3 and the spatial kernel w lives on a cube
Omega = [-W, W]^3.  With the same separable kernels, w(a, b, c) =
w1(a) w1(b) w1(c) (the box of eq. spatial_kernel2 or the Gaussian of eq.
spatial_kernel1 along each axis), eq. (BF), eq. (GPA) and Algorithm 2 keep
their form; only the spatial filtering of eq. (spatialFiltering) runs over
three axes.  The normalised centre weight of Prop. (accuracy) becomes
w(0) = (w1(0) / sum_a w1(a))^3.

Volumes are (D, H, W) arrays (slice, row, column); the border reading is
the zero extension of ``oracle.bf``, or reflection about every face (the
``_mirror`` forms, as ``oracle.mirror`` for images).
"""
from __future__ import annotations

import numpy as np

from .bf import range_kernel
from . import gpa as _gpa
from .gpa import phi, phi_wide


def _shifted(pad: np.ndarray, W: int, a: int, b: int, c: int, shape) -> np.ndarray:
    D, H, Wd = shape
    return pad[W - a:W - a + D, W - b:W - b + H, W - c:W - c + Wd]


def direct_bf(f: np.ndarray, w1: np.ndarray, sigma_r: float) -> np.ndarray:
    """eq. (BF) on a volume with w = w1 x w1 x w1."""
    f = np.asarray(f, dtype=np.float64)
    W = len(w1) // 2
    pad = np.pad(f, W)
    valid = np.pad(np.ones_like(f), W)
    num = np.zeros_like(f)
    den = np.zeros_like(f)
    for a in range(-W, W + 1):
        for b in range(-W, W + 1):
            for c in range(-W, W + 1):
                sh = _shifted(pad, W, a, b, c, f.shape)
                ok = _shifted(valid, W, a, b, c, f.shape)
                k = w1[W + a] * w1[W + b] * w1[W + c] * range_kernel(sh - f, sigma_r) * ok
                num += k * sh
                den += k
    return num / den


def gpa_pairwise(f: np.ndarray, w1: np.ndarray, sigma_r: float, N: int, center: float,
                 wide: bool = False) -> np.ndarray:
    """eq. (GPA) on the centred volume, pair by pair (wide: phi in log space,
    ``oracle.gpa.phi_wide``, finite for T / sigma_r up to 37.4)."""
    ph = phi_wide if wide else phi
    h = np.asarray(f, dtype=np.float64) - center
    W = len(w1) // 2
    pad = np.pad(h, W)
    valid = np.pad(np.ones_like(h), W)
    num = np.zeros_like(h)
    den = np.zeros_like(h)
    for a in range(-W, W + 1):
        for b in range(-W, W + 1):
            for c in range(-W, W + 1):
                sh = _shifted(pad, W, a, b, c, h.shape)
                ok = _shifted(valid, W, a, b, c, h.shape)
                k = w1[W + a] * w1[W + b] * w1[W + c] * ph(sh, h, sigma_r, N) * ok
                num += k * sh
                den += k
    return num / den + center


def spatial_filter(F: np.ndarray, w1: np.ndarray) -> np.ndarray:
    """eq. (spatialFiltering) with w = w1 x w1 x w1 over the zero-extended
    volume: one shifted sum per axis."""
    out = np.asarray(F, dtype=np.float64)
    W = len(w1) // 2
    for axis in range(3):
        L = out.shape[axis]
        acc = np.zeros_like(out)
        for a in range(-W, W + 1):
            lo, hi = max(0, a), min(L, L + a)
            if hi <= lo:
                continue
            dst = [slice(None)] * 3
            src = [slice(None)] * 3
            dst[axis] = slice(lo, hi)
            src[axis] = slice(lo - a, hi - a)
            acc[tuple(dst)] += w1[W + a] * out[tuple(src)]
        out = acc
    return out


def gpa_alg2(f: np.ndarray, w1: np.ndarray, sigma_r: float, N: int, T: float) -> np.ndarray:
    """Eqs. (P), (Q), (PbyQ) on a volume: the sums of ``oracle.gpa.gpa_sums``
    with ``spatial_filter`` above (three axes) as eq. (spatialFiltering)."""
    return _gpa.gpa_sums(f, lambda F: spatial_filter(F, w1), sigma_r, N, T)[0]


def _reflect_pad(f: np.ndarray, W: int) -> np.ndarray:
    return np.pad(np.asarray(f, dtype=np.float64), W, mode="symmetric")


def direct_bf_mirror(f: np.ndarray, w1: np.ndarray, sigma_r: float) -> np.ndarray:
    """eq. (BF) on the volume extended by reflection about every face (edge
    samples repeated): the zero-extension filter on the reflect-padded volume,
    centre crop (every window then lies inside the padding)."""
    W = len(w1) // 2
    D, H, Wd = np.shape(f)
    return direct_bf(_reflect_pad(f, W), w1, sigma_r)[W:W + D, W:W + H, W:W + Wd]


def gpa_pairwise_mirror(f: np.ndarray, w1: np.ndarray, sigma_r: float, N: int, center: float,
                        wide: bool = False) -> np.ndarray:
    """eq. (GPA) pair by pair on the reflected extension of the volume."""
    W = len(w1) // 2
    D, H, Wd = np.shape(f)
    return gpa_pairwise(_reflect_pad(f, W), w1, sigma_r, N, center, wide=wide)[W:W + D, W:W + H, W:W + Wd]


def gpa_alg2_mirror(f: np.ndarray, w1: np.ndarray, sigma_r: float, N: int, T: float) -> np.ndarray:
    """Algorithm 2 on the reflected extension (the auxiliary images are
    pointwise in f, so extending f extends them)."""
    W = len(w1) // 2
    D, H, Wd = np.shape(f)
    return gpa_alg2(_reflect_pad(f, W), w1, sigma_r, N, T)[W:W + D, W:W + H, W:W + Wd]


def w0(w1: np.ndarray) -> float:
    """Normalised centre weight of w1 x w1 x w1."""
    w1 = np.asarray(w1, dtype=np.float64)
    return float((w1[len(w1) // 2] / w1.sum()) ** 3)
