"""Pins for oracle.mirror (the reflecting-border reading): the spatial filter
against scipy.ndimage (mode 'reflect'), the direct filter against a brute
force that indexes the reflection explicitly, the reflection index against
numpy.pad, Algorithm 2 against the pair-by-pair form, and constants."""
import numpy as np
import pytest
from scipy import ndimage

import synthimg
from oracle import kernels as K
from oracle import mirror as M


@pytest.mark.parametrize("n,W", [(5, 2), (4, 7), (1, 3), (9, 9)])
def test_reflect_index_matches_pad(n, W):
    x = np.arange(n, dtype=float) * 3.0 + 1.0
    ref = np.pad(x, W, mode="symmetric")
    assert np.array_equal(x[M.reflect_index(np.arange(-W, n + W), n)], ref)


@pytest.mark.parametrize("kind,kw", [(K.BOX, dict(W=3)), (K.GAUSS, dict(sigma_s=2.0))])
@pytest.mark.parametrize("shape", [(12, 17), (3, 20), (2, 2)])
def test_spatial_filter_matches_library(kind, kw, shape):
    F = synthimg.gen2(*shape, 5)
    w1 = K.taps1d(kind, **kw)
    ref = ndimage.correlate1d(ndimage.correlate1d(F, w1, axis=0, mode="reflect"), w1, axis=1, mode="reflect")
    assert np.allclose(M.spatial_filter(F, w1), ref, rtol=0, atol=1e-9)


def _bf_bruteforce(f, w2, sr):
    H, Wd = f.shape
    W = w2.shape[0] // 2
    out = np.empty((H, Wd))
    for r in range(H):
        for c in range(Wd):
            num = den = 0.0
            for a in range(-W, W + 1):
                for b in range(-W, W + 1):
                    rr = int(M.reflect_index(r - a, H))
                    cc = int(M.reflect_index(c - b, Wd))
                    k = w2[W + a, W + b] * np.exp(-(f[rr, cc] - f[r, c]) ** 2 / (2 * sr * sr))
                    num += k * f[rr, cc]
                    den += k
            out[r, c] = num / den
    return out


def test_direct_bf_bruteforce():
    f = synthimg.gen1(6, 8, 6)
    w2 = K.taps2d(K.GAUSS, 1.5)  # W = 5: wider than the image height, several reflections
    assert np.allclose(M.direct_bf(f, w2, 20.0), _bf_bruteforce(f, w2, 20.0), rtol=0, atol=1e-10)


@pytest.mark.parametrize("N", [1, 6, 30])
def test_alg2_equals_pairwise(N):
    f = synthimg.gen2(13, 15, 7)
    w1, w2 = K.taps1d(K.GAUSS, 1.2), K.taps2d(K.GAUSS, 1.2)
    px = np.array([[r, c] for r in range(13) for c in range(15)])
    a = M.gpa_alg2(f, w1, 30.0, N, 127.5)
    b = M.gpa_pairwise_at(f, px, w2, 30.0, N, 127.5).reshape(13, 15)
    assert np.abs(a - b).max() < 1e-8 * max(1.0, np.abs(b).max())


def test_converges_and_keeps_constants():
    f = synthimg.gen1(12, 14, 8)
    w1, w2 = K.taps1d(K.BOX, W=2), K.taps2d(K.BOX, W=2)
    exact = M.direct_bf(f, w2, 30.0)
    assert np.abs(M.gpa_alg2(f, w1, 30.0, 80, 127.5) - exact).max() < 1e-8
    c = np.full((9, 11), 42.0)
    assert np.abs(M.gpa_alg2(c, w1, 10.0, 5, 127.5) - 42.0).max() < 1e-9
