"""Pins for oracle.order: the order-selection rules and kernel-error bounds
(Sec. 2, Prop. upperBound, Prop. LambW, Algorithm 1; Sec. 3, Cor. eps;
Sec. 4 Tables table1 / table2 / orderComp, eq. Nvsdelta)."""
import math

import numpy as np
import pytest

from oracle import kernels as K
from oracle import order as O
from conftest import load_golden


def test_table1_exact_series_newton():
    # Table 1: eps = 1e-3, T = 128.
    for sr, n1, n2, n3 in load_golden("table1_orders.txt"):
        lam = O.lam_of(128.0, sr)
        assert O.chernoff_order(lam, 1e-3) == n1
        assert O.series_order(lam, 1e-3, newton_steps=0) == n2
        assert O.series_order(lam, 1e-3, newton_steps=3) == n3


def test_table_delta_orders():
    # Table "table2": sigma_r = 30, Gaussian sigma_s = 5 and box W = 4.
    wg = K.w0(K.GAUSS, sigma_s=5.0)
    wb = K.w0(K.BOX, W=4)
    for d, ng, nb in load_golden("table_delta_orders.txt"):
        assert O.order_for_delta(d, wg, 127.5, 30.0) == ng
        assert O.order_for_delta(d, wb, 127.5, 30.0) == nb


def test_table_ordercomp():
    wg = K.w0(K.GAUSS, sigma_s=5.0)
    for d, nl, nv in load_golden("table_ordercomp.txt"):
        assert math.ceil(O.nvsdelta(127.5, 30.0, wg, d)) == nv
        got = O.order_for_delta(d, wg, 127.5, 30.0)
        if d == 1e-2:
            # printed 46; exact Lambert W gives 47 (documented mismatch)
            assert got == 47 and nl == 46
        else:
            assert got == nl


def test_nvsdelta_text_example():
    # Sec. 4 text: sigma_r = 50, 3x3 box, T = 128, delta = 0.01 -> about 24.
    w0 = K.w0(K.BOX, W=1)
    assert math.ceil(O.nvsdelta(128.0, 50.0, w0, 0.01)) == 24


def _poisson_tail_brute(N, lam):
    # direct sum of the Poisson pmf, term by term in log space
    s = 0.0
    n = N
    while True:
        t = math.exp(-lam + n * math.log(lam) - math.lgamma(n + 1))
        s += t
        if n > lam and t < 1e-30 * max(s, 1e-300):
            break
        n += 1
    return s


@pytest.mark.parametrize("lam", [0.5, 3.0, 18.06, 72.25, 162.5])
def test_poisson_tail_matches_pmf_sum(lam):
    for N in [1, 2, 5, int(lam) + 1, int(lam) + 10, int(2 * lam) + 20]:
        a = O.poisson_tail(N, lam)
        b = _poisson_tail_brute(N, lam)
        assert a == pytest.approx(b, rel=1e-9, abs=1e-300)


def test_bisection_matches_lambert_w():
    for T in (127.5, 128.0):
        for sr in (8, 10, 12, 15, 20, 30, 40, 50, 60, 69):
            for eps in (1e-1, 1e-3, 1e-6, 1e-9, 1e-10):
                lam = O.lam_of(T, sr)
                assert O.chernoff_order(lam, eps) == O.chernoff_order_bisect(lam, eps)


def test_chernoff_root_is_smallest_integer_satisfying_inequality():
    # eq. (inequality): e^{-lam} (e lam)^N / N^N <= eps, smallest integer N > lam
    def lhs_log(N, lam):
        return -lam + N * (1.0 + math.log(lam)) - N * math.log(N)
    for sr in (10, 20, 30, 50):
        lam = O.lam_of(127.5, sr)
        for eps in (1e-3, 1e-8):
            N = O.chernoff_order(lam, eps)
            assert N > lam
            assert lhs_log(N, lam) <= math.log(eps) + 1e-12
            assert N - 1 <= lam or lhs_log(N - 1, lam) > math.log(eps)
            # the Chernoff bound dominates the exact Poisson tail
            assert O.poisson_tail(N, lam) <= math.exp(lhs_log(N, lam)) * (1 + 1e-9)
            # hence the exact Poisson order never exceeds the Chernoff order
            assert O.poisson_order(lam, eps) <= N


def test_q_negative_branch():
    # eps > e^{-lam} makes q < 0; W0 on (-1/e, 0) still gives the root > lam
    lam = O.lam_of(127.5, 60.0)
    eps = 0.5 * math.exp(-lam) * 10
    p, q = 1 + math.log(lam), -lam - math.log(eps)
    assert q < 0
    assert O.chernoff_order(lam, eps) == O.chernoff_order_bisect(lam, eps)


@pytest.mark.parametrize("sr,N", [(30.0, 40), (30.0, 20), (20.0, 60), (50.0, 15)])
def test_grid_error_below_poisson_bound(sr, N):
    # Prop. (upperBound), checked on a grid of [-T, T]^2 with T = 128
    T = 128.0
    grid = O.kernel_error_max_grid(N, sr, T, n=201)
    bound = O.poisson_tail(N, O.lam_of(T, sr))
    assert grid <= bound * (1 + 1e-9)


def test_bound_same_order_as_error_fig3():
    # Fig. 3 remark: for sigma_r = 30, N = 40, T = 128 the grid supremum of
    # |E| and the bound are of the same order of magnitude.
    T = 128.0
    grid = O.kernel_error_max_grid(40, 30.0, T, n=257)
    bound = O.poisson_tail(40, O.lam_of(T, 30.0))
    assert bound / grid < 10.0


def test_alg1_literal_modes():
    T = 128.0
    assert O.alg1_order(70.0, 1e-3, T) == 10
    assert O.alg1_order(100.0, 1e-9, T) == 10
    # below 30 the literal algorithm refines the series with Newton steps
    for sr in (10, 15, 20, 25):
        assert O.alg1_order(sr, 1e-3, T) == O.chernoff_order(O.lam_of(T, sr), 1e-3)


def test_eps_delta_accuracy_identity():
    # Cor. (eps) inverts Prop. (accuracy): with eps = w0 d / (2T + d) the
    # accuracy bound 2 T eps / (w0 - eps) equals d.
    for w0 in (1.0 / 81, 1.0 / 157.08, 0.3):
        for d in (1e-3, 0.1, 3.0):
            e = O.eps_from_delta(d, w0, 127.5)
            assert O.accuracy_bound(e, w0, 127.5) == pytest.approx(d, rel=1e-12)


def test_workload_orders():
    # orders used by the workloads (T = 127.5, delta = 1e-3)
    def n(kind, sr, **kw):
        return O.order_for_delta(1e-3, K.w0(kind, **kw), 127.5, sr)
    assert n(K.GAUSS, 30.0, sigma_s=3.0) == 48
    assert n(K.BOX, 20.0, W=5) == 84 and n(K.BOX, 40.0, W=5) == 35
    assert n(K.GAUSS, 30.0, sigma_s=5.0) == 49
    assert n(K.BOX, 30.0, W=30) == 52
