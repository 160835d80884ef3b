"""Pins for oracle.recursive (the recursive Gaussian that Sec. 1 and Sec. 3
cite for O(1) filtering): the fit against the Gaussian it approximates, the
recursions against the convolution they stand for (impulse responses and
random lines), the matrix form of the 2-D filter against a brute-force
double loop, Algorithm 2 against the pair-by-pair form, constants, and
convergence to the direct filter.  The deviation from the exact truncated
Gaussian of eq. (spatial_kernel1) is measured and bounded."""
import numpy as np
import pytest

import synthimg
from oracle import bf as B
from oracle import kernels as K
from oracle import recursive as R


def test_fit_approximates_gaussian():
    # Deriche's constants fit exp(-x^2/2) to about 5e-4 of the peak; a wrong
    # digit in any of the eight moves this by far more
    x = np.linspace(0.0, 12.0, 24001)
    h = R.kernel(x, 1.0)
    assert abs(h[0] - 0.9997) < 1e-12
    assert np.abs(h - np.exp(-x * x / 2)).max() < 6e-4
    assert h.min() > -1.5e-4                      # the small negative lobe
    # the sum over the integers tracks sqrt(2 pi) sigma_s
    for s in (3.0, 10.0, 25.0):
        assert R.kernel_sum(s) == pytest.approx(np.sqrt(2 * np.pi) * s, rel=2e-4)


@pytest.mark.parametrize("sigma_s", [0.7, 2.0, 6.5, 25.0])
def test_recursion_impulse_response(sigma_s):
    L = 200
    X = np.zeros((3, L))
    for k, p in enumerate((0, 77, L - 1)):
        X[k, p] = 1.0
    Y = R.iir_filter_lines(X, sigma_s)
    for k, p in enumerate((0, 77, L - 1)):
        ref = R.kernel(np.arange(L) - p, sigma_s)
        assert np.abs(Y[k] - ref).max() < 1e-12 * max(1.0, sigma_s)


@pytest.mark.parametrize("sigma_s", [1.0, 4.0, 30.0])
def test_recursion_equals_convolution(sigma_s):
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, size=(4, 157))
    direct = X @ R.toeplitz(157, sigma_s).T
    assert np.abs(R.iir_filter_lines(X, sigma_s) - direct).max() < 1e-11 * max(1.0, sigma_s)


def test_matrix_filter_bruteforce():
    F = synthimg.gen2(9, 11, 3)
    s = 1.7
    ref = np.zeros_like(F)
    for r in range(9):
        for c in range(11):
            for i in range(9):
                for j in range(11):
                    ref[r, c] += R.kernel(r - i, s) * R.kernel(c - j, s) * F[i, j]
    assert np.abs(R.spatial_filter(F, s) - ref).max() < 1e-9


def test_separable_recursion_matches_matrix_filter():
    F = synthimg.gen1(23, 31, 4)
    s = 3.3
    rows = R.iir_filter_lines(F, s)                 # along each row
    both = R.iir_filter_lines(rows.T, s).T          # then along each column
    assert np.abs(both - R.spatial_filter(F, s)).max() < 1e-8


@pytest.mark.parametrize("N", [1, 5, 25])
def test_alg2_equals_pairwise(N):
    f = synthimg.gen2(12, 14, 6)
    a = R.gpa_alg2(f, 1.5, 30.0, N, 127.5)
    b = R.gpa_pairwise(f, 1.5, 30.0, N, 127.5)
    assert np.abs(a - b).max() < 1e-8 * max(1.0, np.abs(b).max())


def test_constants_and_convergence():
    c = np.full((10, 13), 77.0)
    assert np.abs(R.gpa_alg2(c, 2.0, 10.0, 6, 127.5) - 77.0).max() < 1e-9
    f = synthimg.gen1(14, 15, 7)
    exact = R.direct_bf(f, 2.0, 30.0)
    errs = [np.abs(R.gpa_alg2(f, 2.0, 30.0, N, 127.5) - exact).max() for N in (10, 30, 80)]
    assert errs[0] >= errs[1] >= errs[2] and errs[2] < 1e-8


def test_order_weight():
    for s in (1.0, 5.0, 25.0):
        n = np.arange(-4000, 4001)
        assert R.w0(s) == pytest.approx((R.kernel(0, s) / R.kernel(n, s).sum()) ** 2, rel=1e-12)
        # close to the exact truncated Gaussian's: the fit, plus the 0.27% of mass beyond 3 sigma_s per axis
        assert R.w0(s) == pytest.approx(K.w0("gauss", sigma_s=s), rel=8e-3)


@pytest.mark.parametrize("sigma_s,sigma_r", [(2.0, 20.0), (4.0, 40.0)])
def test_deviation_from_truncated_gaussian(sigma_s, sigma_r):
    # the recursive kernel differs from the exact 2W+1-tap Gaussian by the fit
    # error and the tails beyond W = 3 sigma_s; on 0-255 images the bilateral
    # outputs stay within a small fraction of a grey level
    f = synthimg.gen2(24, 26, 8)
    rec = R.direct_bf(f, sigma_s, sigma_r)
    ex = B.direct_bf(f, K.taps2d("gauss", sigma_s), sigma_r)
    d = np.abs(rec - ex)
    print(f"sigma_s={sigma_s} sigma_r={sigma_r}: max {d.max():.3e} mean {d.mean():.3e}")
    assert d.max() < 1.5 and d.mean() < 0.2


def test_pointwise_matches_full():
    f = synthimg.gen1(19, 23, 9)
    px = np.array([[0, 0], [18, 22], [7, 11], [0, 22], [12, 3]])
    full = R.gpa_alg2(f, 2.5, 25.0, 12, 127.5)
    assert np.allclose(R.gpa_alg2_at(f, px, 2.5, 25.0, 12, 127.5), full[px[:, 0], px[:, 1]], rtol=0, atol=1e-10)
