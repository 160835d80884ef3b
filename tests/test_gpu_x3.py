"""The streamed Gaussian passes with float32 products emulated by three-way
bfloat16 splits (the default) against the plain float32 matrix-core passes
(BF_FLAG_MFMA_FP32) and the FP64 oracle.

Tolerance: max |GPU - oracle| <= 1e-3 on the 0-255 scale, as for every
forward path.  The two arithmetic forms agree to the float32 rounding
level: BETWEEN = 5e-4 bounds the spread of two float32 summation orders at
sigma_r = 10, N = 252 on 4096^2, where the range-safe coefficients of eq.
(P) reach e^{T/sigma_r} and 2.3e-4 was measured (the fused and streamed
float32 paths differ by 2.1e-4 there too)."""
import numpy as np
import pytest

import synthimg
from oracle import gpa as G
from oracle import kernels as K
from oracle import mirror as M

pytestmark = pytest.mark.gpu
TOL = 1e-3
BETWEEN = 5e-4


def _mods():
    import torch
    import paper_1603_08109_amd as P
    assert torch.cuda.is_available()
    return torch, P


def _pair(f, ss, sr, **kw):
    torch, P = _mods()
    H, Wd = f.shape
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    a = P.Plan("gauss", sr, H, Wd, sigma_s=ss, engine="streamed", **kw)
    b = P.Plan("gauss", sr, H, Wd, sigma_s=ss, engine="streamed", mfma_fp32=True, **kw)
    ya, yb = a.forward(x), b.forward(x)
    torch.cuda.synchronize()
    return (ya.cpu().numpy().astype(np.float64), yb.cpu().numpy().astype(np.float64), a,
            x.cpu().numpy().astype(np.float64))


@pytest.mark.parametrize("ss,sr,shape", [(3.0, 30.0, (100, 300)), (10.0, 10.0, (200, 270)),
                                         (25.0, 30.0, (170, 260)), (40.0, 20.0, (150, 300)),
                                         (41.0, 30.0, (130, 280)), (5.0, 50.0, (64, 64))])
def test_split_matches_fp32_and_oracle(ss, sr, shape):
    # W = 9, 30, 75, 120 (the largest split support) and 123 (falls back to float32)
    f = synthimg.gen2(*shape, 91)
    x3, f32, plan, fx = _pair(f, ss, sr)
    ref = G.gpa_alg2(fx, K.taps1d("gauss", ss), sr, plan.info.N, 127.5)
    d3, d32 = np.abs(x3 - ref).max(), np.abs(f32 - ref).max()
    print(f"sigma_s={ss} W={plan.info.W} N={plan.info.N}: split {d3:.3e} fp32 {d32:.3e} "
          f"between {np.abs(x3 - f32).max():.3e}", flush=True)
    assert d3 <= TOL and d32 <= TOL
    assert np.abs(x3 - f32).max() <= BETWEEN


def test_split_full_size_sampled():
    # the 4096^2 bench shape at sigma_s = 25, sigma_r = 10 (N = 252): sampled pixels
    f = synthimg.gen2(4096, 4096, 3000)
    x3, f32, plan, fx = _pair(f, 25.0, 10.0)
    assert np.abs(x3 - f32).max() <= BETWEEN
    px = synthimg.sample_pixels(4096, 4096, 40, plan.info.W, 15, 3002)
    o2 = G.gpa_pairwise_at(fx, px, K.taps2d("gauss", 25.0), 10.0, plan.info.N, 127.5)
    d = np.abs(x3[px[:, 0], px[:, 1]] - o2).max()
    print(f"N={plan.info.N} sampled max {d:.3e}", flush=True)
    assert d <= TOL


@pytest.mark.parametrize("ss", [4.0, 25.0])
def test_split_mirror(ss):
    f = synthimg.gen2(120, 200, 92)
    x3, f32, plan, fx = _pair(f, ss, 30.0, mirror=True)
    ref = M.gpa_alg2(fx, K.taps1d("gauss", ss), 30.0, plan.info.N, 127.5)
    assert np.abs(x3 - ref).max() <= TOL
    assert np.abs(x3 - f32).max() <= BETWEEN


def test_split_saved_state():
    # the adjoint's saved planes from the split passes agree with the float32 ones
    torch, P = _mods()
    f = synthimg.gen2(140, 200, 93)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    a = P.Plan("gauss", 25.0, 140, 200, sigma_s=8.0, grad=True, engine="streamed")
    b = P.Plan("gauss", 25.0, 140, 200, sigma_s=8.0, grad=True, engine="streamed", mfma_fp32=True)
    sa, sb = a.new_saved(), b.new_saved()
    a.forward(x, saved=sa)
    b.forward(x, saved=sb)
    torch.cuda.synchronize()
    for i, (u, v) in enumerate(zip(sa.view(3, -1), sb.view(3, -1))):
        assert (u - v).abs().max().item() <= 1e-4 * u.abs().max().item() + 1e-12, i


@pytest.mark.parametrize("ss,shape", [(2.0, (70, 300)), (15.0, (130, 270)), (21.3, (140, 200)),
                                      (33.3, (230, 150)), (11.0, (300, 170))])
def test_split_every_step_count(ss, shape):
    # the passes are compiled per k-step count S = ceil((16 + 2W) / 32): W = 6 (S = 1), 45 (S = 4,
    # split columns), 64 (S = 5), 100 (S = 7), 33 (S = 3, the split-once column pass from W = 31:
    # three 128-row tiles, the last ragged); the other counts are covered above
    f = synthimg.gen1(*shape, 94)
    x3, f32, plan, fx = _pair(f, ss, 30.0)
    ref = G.gpa_alg2(fx, K.taps1d("gauss", ss), 30.0, plan.info.N, 127.5)
    d3 = np.abs(x3 - ref).max()
    print(f"sigma_s={ss} W={plan.info.W} N={plan.info.N}: split {d3:.3e}", flush=True)
    assert d3 <= TOL
    assert np.abs(x3 - f32).max() <= BETWEEN


def test_split_saved_state_split_columns():
    # W = 45: the split column pass with the adjoint's sums (SAVE), against the float32 passes
    torch, P = _mods()
    f = synthimg.gen2(150, 180, 95)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    a = P.Plan("gauss", 25.0, 150, 180, sigma_s=15.0, grad=True, engine="streamed")
    b = P.Plan("gauss", 25.0, 150, 180, sigma_s=15.0, grad=True, engine="streamed", mfma_fp32=True)
    assert a.info.W == 45
    sa, sb = a.new_saved(), b.new_saved()
    ya, yb = a.forward(x, saved=sa), b.forward(x, saved=sb)
    torch.cuda.synchronize()
    assert (ya - yb).abs().max().item() <= BETWEEN
    for i, (u, v) in enumerate(zip(sa.view(3, -1), sb.view(3, -1))):
        assert (u - v).abs().max().item() <= 1e-4 * u.abs().max().item() + 1e-12, i
