"""Pins for oracle.volume (the video/volume extension named in Sec. 1 and
Sec. 5): the 3-axis filter against scipy.ndimage with the full 3-D kernel,
the direct filter against a voxel-by-voxel brute force, Algorithm 2 against
the pair-by-pair form, one-slice volumes against the 2-D oracle, constants
and convergence."""
import numpy as np
import pytest
from scipy import ndimage

import synthimg
from oracle import bf as B
from oracle import gpa as G
from oracle import kernels as K
from oracle import volume as V


def _vol(D, H, W, seed):
    return np.stack([synthimg.gen2(H, W, seed + d) for d in range(D)])


@pytest.mark.parametrize("kind,kw", [(K.BOX, dict(W=2)), (K.GAUSS, dict(sigma_s=1.3))])
def test_filter_matches_library(kind, kw):
    F = _vol(5, 7, 9, 1)
    w1 = K.taps1d(kind, **kw)
    w3 = w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
    ref = ndimage.correlate(F, w3, mode="constant")
    assert np.allclose(V.spatial_filter(F, w1), ref, rtol=0, atol=1e-9)


def test_direct_bf_bruteforce():
    f = _vol(3, 4, 5, 2)
    w1 = K.taps1d(K.GAUSS, sigma_s=0.8)
    W = len(w1) // 2
    D, H, Wd = f.shape
    ref = np.empty_like(f)
    for d in range(D):
        for r in range(H):
            for c in range(Wd):
                num = den = 0.0
                for a in range(-W, W + 1):
                    for b in range(-W, W + 1):
                        for e in range(-W, W + 1):
                            dd, rr, cc = d - a, r - b, c - e
                            if 0 <= dd < D and 0 <= rr < H and 0 <= cc < Wd:
                                k = w1[W + a] * w1[W + b] * w1[W + e] * np.exp(
                                    -(f[dd, rr, cc] - f[d, r, c]) ** 2 / (2 * 25.0 ** 2))
                                num += k * f[dd, rr, cc]
                                den += k
                ref[d, r, c] = num / den
    assert np.allclose(V.direct_bf(f, w1, 25.0), ref, rtol=0, atol=1e-10)


@pytest.mark.parametrize("N", [1, 6, 30])
def test_alg2_equals_pairwise(N):
    f = _vol(4, 6, 7, 3)
    w1 = K.taps1d(K.GAUSS, sigma_s=1.0)
    a = V.gpa_alg2(f, w1, 30.0, N, 127.5)
    b = V.gpa_pairwise(f, w1, 30.0, N, 127.5)
    assert np.abs(a - b).max() < 1e-8 * max(1.0, np.abs(b).max())


@pytest.mark.parametrize("kind,kw", [(K.BOX, dict(W=2)), (K.GAUSS, dict(sigma_s=1.5))])
def test_single_slice_is_the_2d_filter(kind, kw):
    # D = 1: the depth taps other than the centre meet zero extension and the
    # centre weight cancels in the ratio
    f = synthimg.gen1(11, 13, 4)
    w1 = K.taps1d(kind, **kw)
    for N in (3, 20):
        assert np.allclose(V.gpa_alg2(f[None], w1, 25.0, N, 127.5)[0], G.gpa_alg2(f, w1, 25.0, N, 127.5),
                           rtol=0, atol=1e-9)
    assert np.allclose(V.direct_bf(f[None], w1, 25.0)[0], B.direct_bf(f, np.outer(w1, w1), 25.0),
                       rtol=0, atol=1e-10)


def test_constants_and_convergence():
    c = np.full((3, 5, 6), 201.0)
    w1 = K.taps1d(K.BOX, W=1)
    assert np.abs(V.gpa_alg2(c, w1, 10.0, 5, 127.5) - 201.0).max() < 1e-9
    f = _vol(4, 5, 6, 5)
    exact = V.direct_bf(f, w1, 30.0)
    errs = [np.abs(V.gpa_alg2(f, w1, 30.0, N, 127.5) - exact).max() for N in (10, 30, 80)]
    assert errs[0] >= errs[1] >= errs[2] and errs[2] < 1e-8


def test_order_weight():
    w1 = K.taps1d(K.GAUSS, sigma_s=2.0)
    assert V.w0(w1) == pytest.approx(K.w0("gauss", sigma_s=2.0) ** 1.5, rel=1e-12)


def _reflect(i, n):
    # reflection about the faces with the edge sample repeated: period 2n
    m = i % (2 * n)
    return m if m < n else 2 * n - 1 - m


def test_mirror_direct_bruteforce():
    # D = 2 and H = 3 below W = 2.. so the reflection wraps more than once
    f = _vol(2, 3, 5, 6)
    w1 = K.taps1d(K.GAUSS, sigma_s=0.8)
    W = len(w1) // 2
    D, H, Wd = f.shape
    ref = np.empty_like(f)
    for d in range(D):
        for r in range(H):
            for c in range(Wd):
                num = den = 0.0
                for a in range(-W, W + 1):
                    for b in range(-W, W + 1):
                        for e in range(-W, W + 1):
                            v = f[_reflect(d - a, D), _reflect(r - b, H), _reflect(c - e, Wd)]
                            k = w1[W + a] * w1[W + b] * w1[W + e] * np.exp(-(v - f[d, r, c]) ** 2 / (2 * 20.0 ** 2))
                            num += k * v
                            den += k
                ref[d, r, c] = num / den
    assert np.allclose(V.direct_bf_mirror(f, w1, 20.0), ref, rtol=0, atol=1e-10)


@pytest.mark.parametrize("N", [2, 12, 40])
def test_mirror_alg2_equals_pairwise(N):
    f = _vol(3, 5, 6, 7)
    w1 = K.taps1d(K.BOX, W=2)
    a = V.gpa_alg2_mirror(f, w1, 30.0, N, 127.5)
    b = V.gpa_pairwise_mirror(f, w1, 30.0, N, 127.5)
    assert np.abs(a - b).max() < 1e-8 * max(1.0, np.abs(b).max())


def test_mirror_single_slice_and_limits():
    # D = 1: every depth tap reads the same slice, so the weights factor out and
    # the result is the 2-D mirror filter; constants stay; large N meets eq. (BF)
    from oracle import mirror as M
    f = synthimg.gen1(9, 11, 8)
    w1 = K.taps1d(K.GAUSS, sigma_s=1.2)
    assert np.allclose(V.direct_bf_mirror(f[None], w1, 25.0)[0], M.direct_bf(f, np.outer(w1, w1), 25.0),
                       rtol=0, atol=1e-10)
    assert np.abs(V.gpa_alg2_mirror(np.full((2, 4, 5), 77.0), w1, 10.0, 6, 127.5) - 77.0).max() < 1e-9
    g = _vol(3, 4, 6, 9)
    exact = V.direct_bf_mirror(g, w1, 30.0)
    assert np.abs(V.gpa_alg2_mirror(g, w1, 30.0, 80, 127.5) - exact).max() < 1e-8


def test_pairwise_wide_forms():
    # phi in log space: the plain pair-by-pair form where that is finite, and the direct
    # filter within the accuracy bound at sigma_r = 4 (lambda = 1016), on the zero and
    # the reflected extension
    f = _vol(3, 5, 6, 10)
    w1 = K.taps1d(K.GAUSS, sigma_s=0.8)
    a = V.gpa_pairwise(f, w1, 8.0, 300, 127.5)
    b = V.gpa_pairwise(f, w1, 8.0, 300, 127.5, wide=True)
    assert np.abs(a - b).max() < 1e-9
    from oracle import order as O
    eps = V.w0(w1) * 1e-3 / (2 * 127.5 + 1e-3)
    N = O.chernoff_order(O.lam_of(127.5, 4.0), eps)
    assert np.abs(V.gpa_pairwise(f, w1, 4.0, N, 127.5, wide=True) - V.direct_bf(f, w1, 4.0)).max() <= 1e-3
    g = _vol(2, 4, 5, 11)
    assert np.abs(V.gpa_pairwise_mirror(g, w1, 4.0, N, 127.5, wide=True) - V.direct_bf_mirror(g, w1, 4.0)).max() <= 1e-3
