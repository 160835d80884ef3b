"""The bilateral filter and its Gaussian-polynomial approximation with a
reflecting (mirror) border, in float64.  Test infrastructure only.

The paper leaves the border open (Sec. 1 defines eq. BF on the image and the
window Omega may leave it); the default reading here is zero extension
(``oracle.bf``).  This module is the alternative reading: the image is
extended by reflection about its edges, repeating the edge sample
(... c b a | a b c d | d c b ...), so every pixel has a full window and
sum_{j in Omega} w(j) is the same everywhere.

Implementation: reflect-pad the image by W on each side (``numpy.pad`` mode
'symmetric', which repeats the reflection for W beyond the image size) and
run the zero-extension filters of ``oracle.bf`` / ``oracle.gpa`` on the
padded image; every output pixel's window then lies inside the padding, so
the zero border never acts, and the centre crop is the mirror-border result.
"""
from __future__ import annotations

import numpy as np

from . import bf as _bf
from . import gpa as _gpa


def reflect_index(i: np.ndarray, n: int) -> np.ndarray:
    """Index of the reflected extension: period 2n, edge samples repeated."""
    m = np.mod(np.asarray(i), 2 * n)
    return np.where(m < n, m, 2 * n - 1 - m)


def _pad(f: np.ndarray, W: int) -> np.ndarray:
    return np.pad(np.asarray(f, dtype=np.float64), W, mode="symmetric")


def spatial_filter(F: np.ndarray, w1: np.ndarray) -> np.ndarray:
    """eq. (spatialFiltering) with the separable kernel w1 x w1 on the reflected extension."""
    W = len(w1) // 2
    H, Wd = np.shape(F)
    return _gpa.spatial_filter(_pad(F, W), w1)[W:W + H, W:W + Wd]


def direct_bf(f: np.ndarray, w2: np.ndarray, sigma_r: float) -> np.ndarray:
    """eq. (BF) with the reflected extension of f."""
    W = w2.shape[0] // 2
    H, Wd = np.shape(f)
    return _bf.direct_bf(_pad(f, W), w2, sigma_r)[W:W + H, W:W + Wd]


def gpa_alg2(f: np.ndarray, w1: np.ndarray, sigma_r: float, N: int, T: float) -> np.ndarray:
    """Algorithm 2 with the reflected extension of the auxiliary images (they
    are pointwise in f, so extending f extends them)."""
    W = len(w1) // 2
    H, Wd = np.shape(f)
    return _gpa.gpa_alg2(_pad(f, W), w1, sigma_r, N, T)[W:W + H, W:W + Wd]


def gpa_pairwise_at(f: np.ndarray, pixels: np.ndarray, w2: np.ndarray, sigma_r: float, N: int,
                    center: float, wide: bool = False) -> np.ndarray:
    """eq. (GPA) with the reflected extension, at the listed (row, col) pixels
    (wide: phi in log space, ``oracle.gpa.phi_wide``)."""
    W = w2.shape[0] // 2
    return _gpa.gpa_pairwise_at(_pad(f, W), np.asarray(pixels) + W, w2, sigma_r, N, center, wide=wide)


def gpa_pairwise(f: np.ndarray, w2: np.ndarray, sigma_r: float, N: int, center: float,
                 wide: bool = False) -> np.ndarray:
    """eq. (GPA) pair by pair with the reflected extension (wide: ``phi_wide``)."""
    W = w2.shape[0] // 2
    H, Wd = np.shape(f)
    return _gpa.gpa_pairwise(_pad(f, W), w2, sigma_r, N, center, wide=wide)[W:W + H, W:W + Wd]
