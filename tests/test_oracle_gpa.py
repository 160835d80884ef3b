"""Pins for oracle.gpa: eq. (GaussPolynomial), eq. (GPA) and Algorithm 2
(Sec. 2-3, App. B) against closed forms, library routines, brute force, the
accuracy bound of Prop. (accuracy) and the saturation seen in Table table1."""
import math

import numpy as np
import pytest
from scipy import ndimage
from scipy.special import gammainc

import synthimg
from oracle import bf as B
from oracle import gpa as G
from oracle import kernels as K
from oracle import order as O
from conftest import load_golden

KERNELS = [(K.BOX, dict(W=2)), (K.GAUSS, dict(sigma_s=1.5)), (K.GAUSS, dict(sigma_s=3.0))]


def test_phi_tail_closed_form():
    # E_N(t, tau) = g(t - tau) * P(N, s) for s = tau t / sigma_r^2 >= 0,
    # since sum_{n >= N} s^n/n! = e^s P(N, s) (regularised incomplete gamma).
    sr = 30.0
    t = np.linspace(0.5, 128, 37)[:, None]
    tau = np.linspace(0.25, 128, 41)[None, :]
    s = t * tau / sr ** 2
    for N in (1, 5, 20, 40):
        ref = np.exp(-((t - tau) ** 2) / (2 * sr ** 2)) * gammainc(N, s)
        assert np.allclose(G.kernel_error(t, tau, sr, N), ref, rtol=1e-9, atol=1e-13)


def test_phi_converges_to_range_kernel():
    # eq. (asymp2): phi_N -> g(t - tau) pointwise
    t, tau = np.meshgrid(np.linspace(-127.5, 127.5, 31), np.linspace(-127.5, 127.5, 29))
    g = np.exp(-((t - tau) ** 2) / (2 * 20.0 ** 2))
    assert np.abs(G.phi(t, tau, 20.0, 200) - g).max() < 1e-12


def _gpa_bruteforce(f, w2, sr, N, c):
    H, Wd = f.shape
    W = w2.shape[0] // 2
    out = np.zeros_like(f)
    for r in range(H):
        for cc in range(Wd):
            tau = f[r, cc] - c
            num = den = 0.0
            for a in range(-W, W + 1):
                for b in range(-W, W + 1):
                    rr, c2 = r - a, cc - b
                    if 0 <= rr < H and 0 <= c2 < Wd:
                        t = f[rr, c2] - c
                        poly = sum((tau * t / sr ** 2) ** n / math.factorial(n) for n in range(N))
                        ph = math.exp(-(t * t + tau * tau) / (2 * sr * sr)) * poly
                        num += w2[W + a, W + b] * ph * t
                        den += w2[W + a, W + b] * ph
            out[r, cc] = num / den + c
    return out


def test_pairwise_bruteforce_tiny():
    f = synthimg.gen1(7, 8, 2)
    w2 = K.taps2d(K.GAUSS, sigma_s=1.0)
    assert np.allclose(G.gpa_pairwise(f, w2, 30.0, 12, 127.5),
                       _gpa_bruteforce(f, w2, 30.0, 12, 127.5), atol=1e-10)


@pytest.mark.parametrize("kind,kw", KERNELS)
@pytest.mark.parametrize("N", [1, 3, 17, 48])
def test_alg2_equals_pairwise(kind, kw, N):
    # App. B: Algorithm 2 computes eq. (GPA) exactly
    f = synthimg.gen2(24, 21, 31)
    w1, w2 = K.taps1d(kind, **kw), K.taps2d(kind, **kw)
    a = G.gpa_alg2(f, w1, 30.0, N, 127.5)
    p = G.gpa_pairwise(f, w2, 30.0, N, 127.5)
    assert np.abs(a - p).max() < 1e-9


@pytest.mark.parametrize("sr,N", [(10.0, 250), (50.0, 30)])
def test_alg2_equals_pairwise_extremes(sr, N):
    f = synthimg.gen2(20, 20, 41)
    kind, kw = K.GAUSS, dict(sigma_s=1.5)
    a = G.gpa_alg2(f, K.taps1d(kind, **kw), sr, N, 127.5)
    p = G.gpa_pairwise(f, K.taps2d(kind, **kw), sr, N, 127.5)
    assert np.all(np.isfinite(a)) and np.abs(a - p).max() < 1e-8


@pytest.mark.parametrize("kind,kw", KERNELS)
@pytest.mark.parametrize("N", [1, 4, 30])
def test_constant_image_fixed_point(kind, kw, N):
    f = np.full((15, 12), 201.0)
    assert np.allclose(G.gpa_alg2(f, K.taps1d(kind, **kw), 25.0, N, 127.5), 201.0, atol=1e-9)


@pytest.mark.parametrize("kind,kw", KERNELS)
def test_order_one_closed_form(kind, kw):
    # N = 1: P/Q = sigma_r (w*F_1)/(w*F_0): the centred image averaged with
    # weights w(j) exp(-h(i-j)^2 / 2 sigma_r^2); computed with library correlation
    f = synthimg.gen1(19, 22, 5)
    sr, c = 35.0, 127.5
    h = f - c
    E = np.exp(-h * h / (2 * sr * sr))
    w2 = K.taps2d(kind, **kw)
    ref = ndimage.correlate(E * h, w2, mode="constant") / ndimage.correlate(E, w2, mode="constant") + c
    assert np.allclose(G.gpa_alg2(f, K.taps1d(kind, **kw), sr, 1, c), ref, atol=1e-10)


@pytest.mark.parametrize("shape", [(17, 26), (3, 3), (1, 9), (8, 1), (1, 1)])
def test_spatial_filter_matches_library(shape):
    # includes images smaller than the kernel support (zero extension)
    f = synthimg.gen2(*shape, 9)
    for kind, kw in KERNELS:
        w1, w2 = K.taps1d(kind, **kw), K.taps2d(kind, **kw)
        assert np.allclose(G.spatial_filter(f, w1), ndimage.correlate(f, w2, mode="constant"), atol=1e-9)


@pytest.mark.parametrize("kind,kw", [(K.BOX, dict(W=3)), (K.GAUSS, dict(sigma_s=2.0))])
@pytest.mark.parametrize("sr", [20.0, 30.0, 45.0])
def test_accuracy_bound_holds(kind, kw, sr):
    # Prop. (accuracy) with ||E|| from Prop. (upperBound); T = 127.5, c = T,
    # inputs in [0, 255].  Zero extension keeps sum w <= 1 after
    # normalisation, so the proof of App. C carries over at the border.
    f = synthimg.gen2(26, 26, int(sr))
    w1, w2 = K.taps1d(kind, **kw), K.taps2d(kind, **kw)
    exact = B.direct_bf(f, w2, sr)
    w0 = K.w0(kind, **kw)
    lam = O.lam_of(127.5, sr)
    for N in range(max(2, int(lam)), int(lam) + 40, 4):
        E = O.poisson_tail(N, lam)
        bound = O.accuracy_bound(E, w0, 127.5)
        err = np.abs(G.gpa_alg2(f, w1, sr, N, 127.5) - exact).max()
        assert err <= bound * (1 + 1e-9) + 1e-10


def test_planned_order_meets_delta():
    # Cor. (eps): N from delta = 1e-3 gives max error <= 1e-3 (workload-1 setting)
    f = synthimg.gen1(64, 64, 1000)
    kind, kw = K.GAUSS, dict(sigma_s=3.0)
    N = O.order_for_delta(1e-3, K.w0(kind, **kw), 127.5, 30.0)
    assert N == 48
    err = np.abs(G.gpa_alg2(f, K.taps1d(kind, **kw), 30.0, N, 127.5)
                 - B.direct_bf(f, K.taps2d(kind, **kw), 30.0)).max()
    assert err <= 1e-3


def test_error_saturates_like_table_exp4():
    # Table table1: error falls steadily with N up to N = 60 and is flat
    # (float64 floor) beyond; here on a synthetic 40x40 image.
    gold = load_golden("table_exp4_saturation.txt")
    f = synthimg.gen1(40, 40, 77)
    for kind, kw, col in [(K.GAUSS, dict(sigma_s=5.0), 1), (K.BOX, dict(W=4), 2)]:
        exact = B.direct_bf(f, K.taps2d(kind, **kw), 30.0)
        errs = [np.abs(G.gpa_alg2(f, K.taps1d(kind, **kw), 30.0, int(row[0]), 127.5) - exact).max()
                for row in gold]
        paper = [row[col] for row in gold]
        # same monotone shape up to N = 60
        assert all(errs[i + 1] < errs[i] for i in range(5))
        assert all(paper[i + 1] < paper[i] for i in range(5))
        # flat floor from N = 60 on, far below the delta = 1e-3 target
        assert max(errs[5:]) < 1e-9
        assert max(errs[5:]) / min(errs[5:]) < 10.0


def test_pairwise_at_matches_full():
    f = synthimg.gen2(30, 28, 3)
    w2 = K.taps2d(K.BOX, W=3)
    full = G.gpa_pairwise(f, w2, 30.0, 20, 127.5)
    px = synthimg.sample_pixels(30, 28, 40, 3, 20, 2)
    assert np.allclose(G.gpa_pairwise_at(f, px, w2, 30.0, 20, 127.5), full[px[:, 0], px[:, 1]], atol=1e-11)
