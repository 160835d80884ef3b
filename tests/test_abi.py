"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and its host-only planning (bf_order) agrees with the
oracle's order rules and reports status codes as documented."""
import math
import os
import re

import numpy as np

import pytest

from oracle import kernels as K
from oracle import order as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1603_08109_amd import _lib as L
    return L, L.load()


def test_exports_every_declared_symbol():
    L, lib = _lib()
    header = open(os.path.join(ROOT, "include", "bf_gpa.h")).read()
    names = set(re.findall(r"^\s*(?:int|const char\*)\s+(bf_\w+)\s*\(", header, re.M))
    assert {"bf_plan", "bf_forward", "bf_backward", "bf_batch_plan", "bf_batch_forward"} <= names
    for n in names:
        assert hasattr(lib, n), n
    assert set(L.SIGNATURES) == names


def test_version_and_status_strings():
    import paper_1603_08109_amd as P
    L, lib = _lib()
    assert "gfx950" in P.version()
    for code in (0, -1, -2, -3, -4, 1):
        assert lib.bf_status_string(code)


@pytest.mark.parametrize("kind,kw", [("box", dict(W=4)), ("box", dict(W=30)),
                                     ("gauss", dict(sigma_s=3.0)), ("gauss", dict(sigma_s=5.0)),
                                     ("gauss", dict(sigma_s=25.0))])
def test_order_matches_oracle(kind, kw):
    import paper_1603_08109_amd as P
    w0 = K.w0(kind, **kw)
    for sr in (10.0, 12.5, 20.0, 30.0, 47.0, 60.0, 90.0):
        for d in (1e-3, 1e-2, 0.1, 1.0, 3.0):
            info = P.bf_order(kind, sr, delta=d, **kw)
            assert info.N == O.order_for_delta(d, w0, 127.5, sr), (sr, d)
            assert info.w0 == pytest.approx(w0, rel=1e-12)
            assert info.eps == pytest.approx(O.eps_from_delta(d, w0, 127.5), rel=1e-12)
            lam = O.lam_of(127.5, sr)
            assert info.kernel_bound == pytest.approx(O.poisson_tail(info.N, lam), rel=1e-6, abs=1e-300)
            assert info.guaranteed_delta <= d * (1 + 1e-9)


def test_poisson_and_alg1_rules():
    import paper_1603_08109_amd as P
    for sr in (15.0, 30.0, 50.0):
        lam = O.lam_of(127.5, sr)
        w0 = K.w0("box", W=4)
        eps = O.eps_from_delta(0.1, w0, 127.5)
        pi = P.bf_order("box", sr, W=4, delta=0.1, n_rule="poisson")
        assert pi.N == O.poisson_order(lam, eps)
        assert pi.N <= P.bf_order("box", sr, W=4, delta=0.1).N
    a = P.bf_order("box", 80.0, W=4, n_rule="alg1")
    assert a.N == 10 and a.status == 1  # sigma_r >= 70: no guarantee
    # Table 1 setting through Algorithm 1 (T = 128, eps = 1e-3 <=> delta with w0 = 1)
    for sr, n in [(20.0, 67), (30.0, 37), (50.0, 19)]:
        d = 1e-3 * 2 * 128.0 / (1.0 - 1e-3)
        got = P.bf_order("box", sr, W=0, T=128.0, delta=d, n_rule="alg1")
        assert got.N == n


def test_status_codes():
    import paper_1603_08109_amd as P
    from paper_1603_08109_amd import _lib as L
    with pytest.raises(L.BFError) as e:
        P.bf_order("box", -1.0, W=3)
    assert e.value.code == L.BF_EINVAL
    with pytest.raises(L.BFError) as e:
        P.bf_order("box", 30.0, W=-2)
    assert e.value.code == L.BF_EINVAL
    with pytest.raises(L.BFError) as e:
        P.bf_order("gauss", 30.0, sigma_s=0.0)
    assert e.value.code == L.BF_EINVAL
    with pytest.raises(L.BFError) as e:
        P.bf_order("box", 5.0, W=3)          # exp(-x^2/2) would underflow float32
    assert e.value.code == L.BF_EUNSUPPORTED
    w = P.bf_order("box", 30.0, W=3, N=5)
    assert w.status == L.BF_WNOGUARANTEE and w.N == 5
    assert math.isinf(w.guaranteed_delta) or w.guaranteed_delta > 1e-3


def test_gaussian_support_rule():
    import paper_1603_08109_amd as P
    for ss, W in [(3.0, 9), (5.0, 15), (25.0, 75), (2.2, 7), (1.0 / 3.0, 1)]:
        assert P.bf_order("gauss", 30.0, sigma_s=ss).W == W
    assert P.bf_order("gauss", 30.0, sigma_s=5.0, W=4).W == 4


def test_engine_selection():
    # host-only: which forward engine a plan would run, and the forcing flags' limits
    import paper_1603_08109_amd as P
    from paper_1603_08109_amd import _lib as L
    kw = dict(height=512, width=512)
    v = P.bf_order("gauss", 30.0, sigma_s=3.0, engine="valu", **kw)
    assert v.path == L.BF_PATH_TILE and v.tile_rows > 0
    s = P.bf_order("gauss", 30.0, sigma_s=3.0, engine="streamed", **kw)
    assert s.path == L.BF_PATH_STREAMED
    assert P.bf_order("gauss", 30.0, sigma_s=25.0, **kw).path == L.BF_PATH_STREAMED  # W = 75
    # the Gaussian takes the streamed passes from W = 16 below 2^22 pixels (W = 15 stays fused); the box
    # keeps its fused tiles below 2^20 pixels
    for H, Wd in ((1, 1), (64, 64), (512, 512), (768, 1024)):
        assert P.bf_order("gauss", 30.0, sigma_s=5.0, height=H, width=Wd).path == L.BF_PATH_TILE  # W = 15
        assert P.bf_order("gauss", 30.0, sigma_s=5.1, height=H, width=Wd).path == L.BF_PATH_STREAMED  # W = 16
        assert P.bf_order("box", 30.0, W=40, height=H, width=Wd).path == L.BF_PATH_TILE
    # from 2^22 pixels the Gaussian goes streamed from W = 17, and from W = 15 with 150 orders or more
    # (sigma_r = 30: N = 49, sigma_r = 10: N = 250)
    big = dict(height=2048, width=2048)
    assert P.bf_order("gauss", 30.0, sigma_s=4.3, **big).path == L.BF_PATH_TILE  # W = 13
    assert P.bf_order("gauss", 10.0, sigma_s=4.3, **big).path == L.BF_PATH_TILE  # W = 13
    assert P.bf_order("gauss", 30.0, W=16, sigma_s=5.2, **big).path == L.BF_PATH_TILE
    assert P.bf_order("gauss", 10.0, W=15, sigma_s=5.0, **big).path == L.BF_PATH_STREAMED
    assert P.bf_order("gauss", 30.0, W=17, sigma_s=5.6, **big).path == L.BF_PATH_STREAMED
    # box strips from 2^20 pixels: from W = 18, and from W = 13 with 150 orders or more
    mid = dict(height=1024, width=1024)
    assert P.bf_order("box", 30.0, W=40, **mid).path == L.BF_PATH_STREAMED
    assert P.bf_order("box", 30.0, W=18, **mid).path == L.BF_PATH_STREAMED
    assert P.bf_order("box", 30.0, W=16, **mid).path == L.BF_PATH_TILE
    assert P.bf_order("box", 10.0, W=13, **mid).path == L.BF_PATH_STREAMED
    assert P.bf_order("box", 10.0, W=12, **mid).path == L.BF_PATH_TILE
    with pytest.raises(L.BFError) as e:
        P.bf_order("gauss", 30.0, sigma_s=3.0, engine="valu", streamed=True, **kw)
    assert e.value.code == L.BF_EINVAL
    # flag bits outside BF_FLAG_* (64 was the removed matrix-core tile) are refused
    import ctypes as C
    from paper_1603_08109_amd import api
    p = api.make_params("gauss", 30.0, sigma_s=3.0, **kw)
    p.flags |= 64
    info = L.bf_plan_info()
    assert L.load().bf_order(C.byref(p), C.byref(info)) == L.BF_EINVAL


def test_recursive_gaussian_planning():
    # host-only: w0 from the fit's closed-form sum, N from the same rule, engine and limits
    import paper_1603_08109_amd as P
    from oracle import recursive as R
    from paper_1603_08109_amd import _lib as L
    for ss in (0.5, 3.0, 25.0, 100.0):
        w0 = R.w0(ss)
        for sr in (10.0, 30.0, 60.0):
            info = P.bf_order("gauss_rec", sr, sigma_s=ss, height=512, width=512)
            assert info.w0 == pytest.approx(w0, rel=1e-10)
            assert info.N == O.order_for_delta(1e-3, w0, 127.5, sr)
            assert info.path == L.BF_PATH_RECURSIVE and info.W == 0
    for bad in (dict(sigma_s=0.3), dict(sigma_s=150.0)):
        with pytest.raises(L.BFError) as e:
            P.bf_order("gauss_rec", 30.0, **bad)
        assert e.value.code == L.BF_EINVAL
    with pytest.raises(L.BFError) as e:
        P.bf_order("gauss_rec", 30.0, sigma_s=3.0, height=9000, width=64)   # lines longer than 8192
    assert e.value.code == L.BF_EUNSUPPORTED
    assert P.bf_order("gauss_rec", 30.0, sigma_s=3.0, height=64, width=8192).path == L.BF_PATH_RECURSIVE


def test_wide_range_planning():
    # host-only: lambda = (T / sigma_r)^2 in (170, 1400] runs the Gaussian on
    # the wide-range streamed path only; every other request there, and any
    # lambda above 1400, is unsupported
    import paper_1603_08109_amd as P
    from paper_1603_08109_amd import _lib as L
    kw = dict(height=256, width=300)
    for sr, ss in [(9.7, 2.0), (6.0, 3.0), (3.41, 1.0), (5.0, 40.0)]:
        info = P.bf_order("gauss", sr, sigma_s=ss, **kw)
        assert info.path == L.BF_PATH_WIDE and info.tile_cols == 0, (sr, ss)
        assert info.lam == pytest.approx((127.5 / sr) ** 2)
        assert info.N == O.order_for_delta(1e-3, K.w0("gauss", sigma_s=ss), 127.5, sr)
        assert P.bf_order("gauss", sr, sigma_s=ss).path == L.BF_PATH_WIDE  # no size needed
    assert P.bf_order("gauss", 9.8, sigma_s=2.0, **kw).path != L.BF_PATH_WIDE      # lambda 169.3
    assert P.bf_order("gauss", 6.0, sigma_s=2.0, mirror=True, **kw).path == L.BF_PATH_WIDE
    assert P.bf_order("gauss", 5.0, sigma_s=2.0, T=60.0, **kw).path != L.BF_PATH_WIDE  # data range
    bad = [dict(kernel="box", W=3), dict(kernel="gauss", sigma_s=2.0, grad=True),
           dict(kernel="gauss", sigma_s=2.0, joint=True),
           dict(kernel="gauss", sigma_s=2.0, engine="valu"),
           dict(kernel="gauss", sigma_s=2.0, mfma_fp32=True), dict(kernel="gauss", sigma_s=41.0),
           dict(kernel="gauss_rec", sigma_s=2.0)]
    for b in bad:
        k = b.pop("kernel")
        with pytest.raises(L.BFError) as e:
            P.bf_order(k, 6.0, **b, **kw)
        assert e.value.code == L.BF_EUNSUPPORTED, (k, b)
    with pytest.raises(L.BFError) as e:
        P.bf_order("gauss", 3.4, sigma_s=2.0, **kw)                    # lambda 1406
    assert e.value.code == L.BF_EUNSUPPORTED
    with pytest.raises(L.BFError) as e:
        P.VolumePlan("box", 6.0, 4, 32, 32, W=1)                      # volumes: the Gaussian only there
    assert e.value.code == L.BF_EUNSUPPORTED


def test_volume_planning_weight():
    # host-side check through the oracle: the 3-D centre weight and its order
    from oracle import volume as V
    w1 = K.taps1d("gauss", sigma_s=2.0)
    assert V.w0(w1) == pytest.approx((w1[len(w1) // 2] / w1.sum()) ** 3, rel=1e-12)
    assert O.order_for_delta(1e-3, V.w0(w1), 127.5, 30.0) >= O.order_for_delta(1e-3, K.w0("gauss", sigma_s=2.0),
                                                                                  127.5, 30.0)


def test_recursive_gaussian_claims_no_guarantee():
    # Prop. (accuracy) assumes w >= 0; Deriche's fit has small negative lobes, so a
    # recursive-Gaussian plan reports the warning and an infinite guaranteed delta
    # (N still follows Cor. eps with the fit's normalised centre weight)
    import paper_1603_08109_amd as P
    from paper_1603_08109_amd import _lib as L
    from oracle import recursive as R
    for ss, sr in [(3.0, 30.0), (25.0, 10.0)]:
        info = P.bf_order("gauss_rec", sr, sigma_s=ss, height=256, width=256)
        assert info.status == L.BF_WNOGUARANTEE
        assert math.isinf(info.guaranteed_delta)
        assert R.kernel(np.arange(0, 8 * int(ss) + 8), ss).min() < 0.0  # the lobes that void the bound
        assert info.w0 == pytest.approx(R.w0(ss), rel=1e-9)
        assert info.N == O.chernoff_order(O.lam_of(127.5, sr), O.eps_from_delta(1e-3, R.w0(ss), 127.5))
