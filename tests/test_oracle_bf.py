"""Pins for oracle.bf (eq. BF, Sec. 1) against properties the definition fixes."""
import math

import numpy as np
import pytest
from scipy import ndimage

import synthimg
from oracle import bf as B
from oracle import kernels as K

KERNELS = [(K.BOX, dict(W=2)), (K.GAUSS, dict(sigma_s=1.5))]


def _bruteforce(f, w2, sr):
    # pure-python loops over pixels and offsets
    H, Wd = f.shape
    W = w2.shape[0] // 2
    out = np.zeros_like(f)
    for r in range(H):
        for c in range(Wd):
            num = den = 0.0
            for a in range(-W, W + 1):
                for b in range(-W, W + 1):
                    rr, cc = r - a, c - b
                    if 0 <= rr < H and 0 <= cc < Wd:
                        k = w2[W + a, W + b] * math.exp(-((f[rr, cc] - f[r, c]) ** 2) / (2 * sr * sr))
                        num += k * f[rr, cc]
                        den += k
            out[r, c] = num / den
    return out


@pytest.mark.parametrize("kind,kw", KERNELS)
def test_bruteforce_tiny(kind, kw):
    f = synthimg.gen1(11, 9, 7)
    w2 = K.taps2d(kind, **kw)
    assert np.allclose(B.direct_bf(f, w2, 25.0), _bruteforce(f, w2, 25.0), rtol=0, atol=1e-11)


@pytest.mark.parametrize("kind,kw", KERNELS)
def test_constant_image(kind, kw):
    f = np.full((13, 17), 93.25)
    assert np.allclose(B.direct_bf(f, K.taps2d(kind, **kw), 20.0), 93.25, atol=1e-12)


@pytest.mark.parametrize("kind,kw", KERNELS)
def test_large_sigma_r_is_spatial_filter(kind, kw):
    # sigma_r -> infinity: g == 1, eq. BF is the spatial filter normalised
    # over the in-image part of Omega (library correlation with zero padding)
    f = synthimg.gen1(20, 23, 3)
    w2 = K.taps2d(kind, **kw)
    num = ndimage.correlate(f, w2, mode="constant", cval=0.0)
    den = ndimage.correlate(np.ones_like(f), w2, mode="constant", cval=0.0)
    assert np.allclose(B.direct_bf(f, w2, 1e7), num / den, rtol=0, atol=1e-7)


def test_small_sigma_r_is_identity():
    rng = np.random.default_rng(5)
    f = rng.permutation(400).reshape(20, 20).astype(np.float64) * 0.6  # distinct levels
    out = B.direct_bf(f, K.taps2d(K.GAUSS, sigma_s=2.0), 1e-2)
    assert np.allclose(out, f, atol=1e-9)


@pytest.mark.parametrize("kind,kw", KERNELS)
def test_affine_covariance_and_centering(kind, kw):
    f = synthimg.gen1(18, 15, 11)
    w2 = K.taps2d(kind, **kw)
    base = B.direct_bf(f, w2, 30.0)
    a, b = 0.37, -12.5
    assert np.allclose(B.direct_bf(a * f + b, w2, a * 30.0), a * base + b, atol=1e-10)
    # Prop. (centering): f_BF = h_BF + t_c
    assert np.allclose(B.direct_bf(f - 127.5, w2, 30.0) + 127.5, base, atol=1e-10)


@pytest.mark.parametrize("kind,kw", KERNELS)
def test_transpose_and_flip(kind, kw):
    f = synthimg.gen1(14, 19, 13)
    w2 = K.taps2d(kind, **kw)
    base = B.direct_bf(f, w2, 30.0)
    assert np.allclose(B.direct_bf(f.T, w2, 30.0), base.T, atol=1e-11)
    assert np.allclose(B.direct_bf(f[::-1, ::-1], w2, 30.0), base[::-1, ::-1], atol=1e-11)


def test_sampled_matches_full():
    f = synthimg.gen2(40, 33, 17)
    w2 = K.taps2d(K.GAUSS, sigma_s=2.0)
    full = B.direct_bf(f, w2, 30.0)
    px = synthimg.sample_pixels(40, 33, 60, 6, 30, 1)
    assert np.allclose(B.direct_bf_at(f, px, w2, 30.0), full[px[:, 0], px[:, 1]], atol=1e-11)


def test_output_is_convex_combination():
    f = synthimg.gen2(30, 30, 21)
    out = B.direct_bf(f, K.taps2d(K.BOX, W=3), 15.0)
    assert out.min() >= f.min() - 1e-9 and out.max() <= f.max() + 1e-9
