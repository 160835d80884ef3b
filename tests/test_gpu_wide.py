"""GPU parity of the wide-range streamed Gaussian (BF_PATH_WIDE: T/sigma_r in
(13, 37.4], float64 per-pixel states) against the FP64 oracle: eq. (GPA)
pair by pair (``oracle.gpa.gpa_pairwise``; with ``wide=True`` its terms are
formed in log space, the only form finite below sigma_r ~ 4.8 on [0, 255]).

Tolerance: max |GPU - oracle| <= 1e-3 on the 0-255 scale, as for every
forward path, oracle in float64 on the float32-rounded input at the same N.
Shapes span one row-pass tile, several tiles with ragged tails, lines of one
pixel, supports W = 3 .. 105 (both register budgets of the split passes),
and the 4096^2 shape at sampled pixels."""
import numpy as np
import pytest

import synthimg
from oracle import bf as B
from oracle import gpa as G
from oracle import kernels as K

pytestmark = pytest.mark.gpu
TOL = 1e-3


def _mods():
    import torch
    import paper_1603_08109_amd as P
    assert torch.cuda.is_available()
    return torch, P


def _forward(f, sr, ss, **kw):
    torch, P = _mods()
    H, Wd = f.shape
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    plan = P.Plan("gauss", sr, H, Wd, sigma_s=ss, **kw)
    assert plan.info.path == P.BF_PATH_WIDE
    out = plan.forward(x)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), plan, x.cpu().numpy().astype(np.float64)


def _report(name, d):
    print(f"{name}: max {np.abs(d).max():.3e} rms {np.sqrt(np.mean(d * d)):.3e}", flush=True)


@pytest.mark.parametrize("ss,sr,shape,seed", [(2.0, 9.5, (40, 56), 1), (2.0, 6.0, (33, 70), 2),
                                              (1.5, 5.0, (48, 64), 3), (3.0, 8.0, (70, 290), 4),
                                              (1.0, 7.0, (20, 300), 5)])
def test_matches_pairwise(ss, sr, shape, seed):
    f = synthimg.gen2(*shape, seed)
    out, plan, fx = _forward(f, sr, ss)
    ref = G.gpa_pairwise(fx, K.taps2d("gauss", sigma_s=ss), sr, plan.info.N, 127.5)
    print(f"sigma_s={ss} sigma_r={sr} {shape}: W={plan.info.W} N={plan.info.N}", flush=True)
    _report("gpu-oracle", out - ref)
    assert np.abs(out - ref).max() <= TOL


def _sample(H, Wd, n, seed):
    rng = np.random.default_rng(seed)
    px = [[0, 0], [0, Wd - 1], [H - 1, 0], [H - 1, Wd - 1], [H // 2, Wd // 2]]
    px += [[int(r), int(c)] for r, c in zip(rng.integers(0, H, n), rng.integers(0, Wd, n))]
    return np.array(px)


@pytest.mark.parametrize("ss,sr,shape,seed", [(2.0, 3.5, (64, 96), 11), (1.0, 4.2, (50, 300), 12),
                                              (15.0, 6.0, (150, 200), 13), (35.0, 8.0, (260, 270), 14)])
def test_sampled_log_space(ss, sr, shape, seed):
    # sigma_r below 4.8 (log-space oracle) and supports W = 45, 105
    f = synthimg.gen2(*shape, seed)
    out, plan, fx = _forward(f, sr, ss)
    px = _sample(*shape, 25, seed)
    ref = G.gpa_pairwise_at(fx, px, K.taps2d("gauss", sigma_s=ss), sr, plan.info.N, 127.5, wide=True)
    got = out[px[:, 0], px[:, 1]]
    print(f"sigma_s={ss} sigma_r={sr} {shape}: W={plan.info.W} N={plan.info.N}", flush=True)
    _report("gpu-oracle", got - ref)
    assert np.abs(got - ref).max() <= TOL


@pytest.mark.parametrize("shape", [(1, 1), (1, 300), (300, 1), (17, 257), (65, 129)])
def test_ragged_and_tiny(shape):
    f = synthimg.gen1(*shape, 21)
    out, plan, fx = _forward(f, 6.0, 2.0)
    ref = G.gpa_pairwise(fx, K.taps2d("gauss", sigma_s=2.0), 6.0, plan.info.N, 127.5)
    assert np.abs(out - ref).max() <= TOL, shape


def test_constants_and_direct_filter():
    # constants are fixed points, also at the ends of the range (|x| = 36.4)
    for v in (0.0, 91.0, 255.0):
        out, _, _ = _forward(np.full((40, 70), v), 3.5, 2.0)
        assert np.abs(out - v).max() <= TOL, v
    # at a small delta the result is the direct filter of eq. (BF)
    f = synthimg.gen1(24, 28, 51)
    out, plan, fx = _forward(f, 4.0, 1.5, delta=1e-5)
    exact = B.direct_bf(fx, K.taps2d("gauss", sigma_s=1.5), 4.0)
    _report(f"gpu-direct N={plan.info.N}", out - exact)
    assert np.abs(out - exact).max() <= TOL


def test_data_range_still_float32():
    # a narrow data range keeps lambda <= 170 at the same sigma_r: the float32 paths
    torch, P = _mods()
    f = 100.0 + 40.0 * synthimg.gen2(30, 40, 61) / 255.0
    plan = P.Plan("gauss", 5.0, 30, 40, sigma_s=2.0, T=20.0, center=120.0)
    assert plan.info.path != P.BF_PATH_WIDE


@pytest.mark.parametrize("ss,sr", [(3.0, 5.0), (25.0, 3.5)])
def test_full_size_sampled(ss, sr):
    f = synthimg.gen2(4096, 4096, 4200)
    out, plan, fx = _forward(f, sr, ss)
    px = np.array([[0, 0], [0, 4095], [4095, 0], [4095, 4095], [2048, 2047], [17, 3001], [3999, 5],
                   [1024, 1024], [77, 4000], [2500, 1]])
    ref = G.gpa_pairwise_at(fx, px, K.taps2d("gauss", sigma_s=ss), sr, plan.info.N, 127.5, wide=True)
    got = out[px[:, 0], px[:, 1]]
    print(f"W={plan.info.W} N={plan.info.N}", flush=True)
    _report("gpu-oracle", got - ref)
    assert np.abs(got - ref).max() <= TOL


@pytest.mark.parametrize("ss,sr,shape", [(2.0, 5.0, (40, 70)), (12.0, 6.0, (90, 120)), (30.0, 8.0, (150, 170))])
def test_mirror_border(ss, sr, shape):
    # the reflecting border on the wide-range passes (W = 6, 36, 90), against eq. (GPA) on the
    # reflected extension, at every pixel of the small image and sampled ones of the larger
    from oracle import mirror as M
    f = synthimg.gen2(*shape, 71)
    out, plan, fx = _forward(f, sr, ss, mirror=True)
    w2 = K.taps2d("gauss", sigma_s=ss)
    if shape[0] * shape[1] <= 4000:
        ref = M.gpa_pairwise(fx, w2, sr, plan.info.N, 127.5, wide=True)
        d = out - ref
    else:
        px = _sample(*shape, 20, 72)
        d = out[px[:, 0], px[:, 1]] - M.gpa_pairwise_at(fx, px, w2, sr, plan.info.N, 127.5, wide=True)
    print(f"sigma_s={ss} sigma_r={sr} W={plan.info.W} N={plan.info.N}", flush=True)
    _report("gpu-oracle", d)
    assert np.abs(d).max() <= TOL


def test_unsupported_and_saved():
    torch, P = _mods()
    plan = P.Plan("gauss", 6.0, 32, 32, sigma_s=2.0)
    x = torch.zeros(32, 32, device="cuda")
    with pytest.raises(P.BFError):
        plan.forward(x, saved=torch.empty(3 * 32 * 32, device="cuda"))
    for kw in (dict(grad=True), dict(mfma_fp32=True)):
        with pytest.raises(P.BFError):
            P.Plan("gauss", 6.0, 32, 32, sigma_s=2.0, **kw)
