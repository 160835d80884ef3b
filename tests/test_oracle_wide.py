"""Pins for oracle.gpa.phi_wide (eq. GaussPolynomial with every term formed in
log space, for lambda = T^2 / sigma_r^2 up to 1400) and the pair-by-pair
filter built on it: the incomplete-gamma closed form for s >= 0, a
600-digit decimal sum for s < 0 (where the alternating partial sums cancel),
the plain ``phi`` wherever its partial sums are finite, and the direct
filter within the accuracy bound of Prop. (accuracy) at sigma_r = 3.5."""
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy.special import gammaincc

import synthimg
from oracle import bf as B
from oracle import gpa as G
from oracle import kernels as K
from oracle import order as O


@pytest.mark.parametrize("sr", [3.5, 5.0])
@pytest.mark.parametrize("N", [1, 40, 900, 1700])
def test_closed_form_nonnegative_s(sr, N):
    # sum_{n < N} s^n / n! = e^s Q(N, s) (regularised upper incomplete gamma),
    # so phi_N = g(t - tau) Q(N, s) for s = t tau / sigma_r^2 >= 0
    t = np.linspace(0.0, 127.5, 23)[:, None]
    tau = np.linspace(0.0, 127.5, 19)[None, :]
    s = t * tau / sr ** 2
    ref = np.exp(-((t - tau) ** 2) / (2 * sr ** 2)) * gammaincc(N, s)
    got = G.phi_wide(t, tau, sr, N)
    assert np.allclose(got, ref, rtol=1e-9, atol=1e-15)
    got = G.phi_wide(-t, -tau, sr, N)  # the same s
    assert np.allclose(got, ref, rtol=1e-9, atol=1e-15)


def _phi_decimal(t, tau, sr, N):
    getcontext().prec = 600
    t, tau, sr = Decimal(repr(t)), Decimal(repr(tau)), Decimal(repr(sr))
    s = t * tau / (sr * sr)
    term, acc = Decimal(1), Decimal(0)
    for n in range(N):
        if n:
            term = term * s / n
        acc += term
    return float((-(t * t + tau * tau) / (2 * sr * sr)).exp() * acc)


@pytest.mark.parametrize("t,tau", [(127.5, -127.5), (100.0, -3.0), (-60.0, 90.5), (-127.5, 20.25), (5.0, -5.0)])
def test_negative_s_high_precision(t, tau):
    # the alternating partial sums reach e^{|s|}; the terms here stay <= 1
    for sr, N in ((3.5, 1400), (4.0, 700), (6.0, 40)):
        ref = _phi_decimal(t, tau, sr, N)
        assert abs(G.phi_wide(t, tau, sr, N) - ref) <= 1e-12, (t, tau, sr, N)


@pytest.mark.parametrize("sr,N", [(30.0, 20), (8.0, 300), (5.0, 700)])
def test_matches_phi_where_finite(sr, N):
    t, tau = np.meshgrid(np.linspace(-127.5, 127.5, 31), np.linspace(-127.5, 127.5, 29))
    a, b = G.phi(t, tau, sr, N), G.phi_wide(t, tau, sr, N)
    assert np.all(np.isfinite(a))
    assert np.abs(a - b).max() <= 1e-12


def test_pairwise_wide_meets_accuracy_bound():
    # sigma_r = 3.5 (lambda = 1327): the planned order keeps eq. (GPA) within
    # the Prop. (accuracy) bound of the direct filter of eq. (BF)
    f = synthimg.gen2(14, 17, 71)
    w2 = K.taps2d(K.GAUSS, sigma_s=1.0)
    sr, T = 3.5, 127.5
    eps = K.w0(K.GAUSS, sigma_s=1.0) * 1e-3 / (2 * T + 1e-3)
    N = O.chernoff_order(O.lam_of(T, sr), eps)
    got = G.gpa_pairwise(f, w2, sr, N, 127.5, wide=True)
    exact = B.direct_bf(f, w2, sr)
    assert np.all(np.isfinite(got))
    assert np.abs(got - exact).max() <= 1e-3
    # and it agrees with the pixel-sampled form
    px = np.array([[0, 0], [13, 16], [7, 8], [3, 15]])
    at = G.gpa_pairwise_at(f, px, w2, sr, N, 127.5, wide=True)
    assert np.abs(at - got[px[:, 0], px[:, 1]]).max() <= 1e-9


def test_mirror_pairwise_wide_meets_accuracy_bound():
    # the reflected extension at sigma_r = 3.5: eq. (GPA) in log space against eq. (BF), and the
    # pixel-sampled form against the full one
    from oracle import mirror as M
    f = synthimg.gen1(12, 15, 73)
    w2 = K.taps2d(K.GAUSS, sigma_s=1.0)
    sr, T = 3.5, 127.5
    eps = K.w0(K.GAUSS, sigma_s=1.0) * 1e-3 / (2 * T + 1e-3)
    N = O.chernoff_order(O.lam_of(T, sr), eps)
    got = M.gpa_pairwise(f, w2, sr, N, 127.5, wide=True)
    assert np.abs(got - M.direct_bf(f, w2, sr)).max() <= 1e-3
    px = np.array([[0, 0], [11, 14], [5, 7]])
    assert np.abs(M.gpa_pairwise_at(f, px, w2, sr, N, 127.5, wide=True) - got[px[:, 0], px[:, 1]]).max() <= 1e-9
