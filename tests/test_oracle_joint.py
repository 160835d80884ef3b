"""Pins for oracle.joint (the cross/joint bilateral filter named in Sec. 1 and
Sec. 5, and its Gaussian-polynomial form): brute force, the plain filter as
the special case guide = input, a library routine for a constant guide, the
two GPA formulations against each other, constants as fixed points, and
convergence to the exact cross filter as N grows."""
import numpy as np
import pytest
from scipy import ndimage

import synthimg
from oracle import bf as B
from oracle import gpa as G
from oracle import joint as J
from oracle import kernels as K

KERNELS = [(K.BOX, dict(W=2)), (K.GAUSS, dict(sigma_s=1.5))]


def _joint_bruteforce(f, h, w2, sr):
    H, Wd = f.shape
    W = w2.shape[0] // 2
    out = np.empty((H, Wd))
    for r in range(H):
        for c in range(Wd):
            num = den = 0.0
            for a in range(-W, W + 1):
                for b in range(-W, W + 1):
                    rr, cc = r - a, c - b
                    if 0 <= rr < H and 0 <= cc < Wd:
                        k = w2[W + a, W + b] * np.exp(-(h[rr, cc] - h[r, c]) ** 2 / (2 * sr * sr))
                        num += k * f[rr, cc]
                        den += k
            out[r, c] = num / den
    return out


def _pair(shape, seed):
    f = synthimg.gen2(*shape, seed)
    h = synthimg.gen1(*shape, seed + 50)
    return f, h


def test_direct_joint_bruteforce_tiny():
    f, h = _pair((7, 9), 1)
    w2 = K.taps2d(K.GAUSS, 1.2)
    assert np.allclose(J.direct_joint_bf(f, h, w2, 25.0), _joint_bruteforce(f, h, w2, 25.0), rtol=0, atol=1e-11)


@pytest.mark.parametrize("kind,kw", KERNELS)
def test_guide_equal_input_is_plain_filter(kind, kw):
    # h = f: the cross filter is eq. (BF), and its 2N-filtering GPA form equals
    # Algorithm 2 (the numerator f = c + sigma_r x shifts the order by one)
    f = synthimg.gen2(20, 23, 2)
    w1, w2 = K.taps1d(kind, **kw), K.taps2d(kind, **kw)
    assert np.allclose(J.direct_joint_bf(f, f, w2, 30.0), B.direct_bf(f, w2, 30.0), rtol=0, atol=1e-10)
    for N in (1, 7, 30):
        a = J.gpa_joint_alg2(f, f, w1, 30.0, N, 127.5)
        b = G.gpa_alg2(f, w1, 30.0, N, 127.5)
        assert np.abs(a - b).max() < 1e-9, N


@pytest.mark.parametrize("kind,kw", KERNELS)
def test_constant_guide_is_normalised_spatial_filter(kind, kw):
    # a flat guide makes every range weight 1: out = (w * f)/(w * 1), zero extension
    f = synthimg.gen2(18, 21, 3)
    h = np.full_like(f, 77.0)
    w2 = K.taps2d(kind, **kw)
    ref = ndimage.correlate(f, w2, mode="constant") / ndimage.correlate(np.ones_like(f), w2, mode="constant")
    assert np.allclose(J.direct_joint_bf(f, h, w2, 20.0), ref, rtol=0, atol=1e-10)
    for N in (1, 10):
        assert np.allclose(J.gpa_joint_alg2(f, h, K.taps1d(kind, **kw), 20.0, N, 127.5), ref, rtol=0, atol=1e-9)


@pytest.mark.parametrize("kind,kw", KERNELS)
@pytest.mark.parametrize("N", [1, 4, 25])
def test_alg2_equals_pairwise(kind, kw, N):
    # the filtering form and the pair-by-pair form of the same approximation
    f, h = _pair((15, 17), 4)
    a = J.gpa_joint_alg2(f, h, K.taps1d(kind, **kw), 35.0, N, 127.5)
    b = J.gpa_joint_pairwise(f, h, K.taps2d(kind, **kw), 35.0, N, 127.5)
    assert np.abs(a - b).max() < 1e-8 * max(1.0, np.abs(b).max())


def test_constant_input_is_fixed_point():
    h = synthimg.gen1(16, 19, 5)
    f = np.full_like(h, 211.25)
    for N in (1, 6, 40):
        out = J.gpa_joint_alg2(f, h, K.taps1d(K.GAUSS, 2.0), 15.0, N, 127.5)
        assert np.abs(out - 211.25).max() < 1e-9


def test_converges_to_cross_filter():
    f, h = _pair((14, 16), 6)
    w1, w2 = K.taps1d(K.GAUSS, 1.5), K.taps2d(K.GAUSS, 1.5)
    exact = J.direct_joint_bf(f, h, w2, 30.0)
    errs = [np.abs(J.gpa_joint_alg2(f, h, w1, 30.0, N, 127.5) - exact).max() for N in (5, 15, 30, 60)]
    assert all(e1 >= e2 * 0.999 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-8


def test_pointwise_matches_full():
    f, h = _pair((13, 18), 7)
    w2 = K.taps2d(K.BOX, W=2)
    px = np.array([[0, 0], [5, 7], [12, 17], [6, 0], [0, 11]])
    full_d = J.direct_joint_bf(f, h, w2, 25.0)
    full_g = J.gpa_joint_pairwise(f, h, w2, 25.0, 12, 127.5)
    assert np.allclose(J.direct_joint_bf_at(f, h, px, w2, 25.0), full_d[px[:, 0], px[:, 1]], rtol=0, atol=1e-12)
    assert np.allclose(J.gpa_joint_pairwise_at(f, h, px, w2, 25.0, 12, 127.5), full_g[px[:, 0], px[:, 1]],
                       rtol=0, atol=1e-12)
