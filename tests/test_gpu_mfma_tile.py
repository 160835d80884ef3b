"""GPU parity of the fused matrix-core Gaussian tile (BF_FLAG_TILE_MFMA)
against the FP64 CPU oracle.

The same tolerance as the other forward paths: max |GPU - oracle| <= 1e-3 on
the 0-255 scale, oracle in float64 on the float32-rounded input at the same
order N.  Shapes cover one tile, several tiles with ragged tails in both
directions, images smaller than the halo, the widest support the tile holds
(W = 45), and the mirror border.  The adjoint run from this engine's saved
state is checked against float64 autograd.
"""
import numpy as np
import pytest

import synthimg
from oracle import bf as B
from oracle import gpa as G
from oracle import grad as GR
from oracle import kernels as K
from oracle import mirror as M

pytestmark = pytest.mark.gpu
TOL = 1e-3
RTOL = 1e-3


def _mods():
    import torch
    import paper_1603_08109_amd as P
    assert torch.cuda.is_available()
    return torch, P


def _forward(f, sr, sigma_s, **kw):
    torch, P = _mods()
    H, Wd = f.shape
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    plan = P.Plan("gauss", sr, H, Wd, sigma_s=sigma_s, engine="mfma", **kw)
    assert plan.info.path == P.BF_PATH_TILE_MFMA
    out = plan.forward(x)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), plan, x.cpu().numpy().astype(np.float64)


def _report(name, d):
    print(f"{name}: max {np.abs(d).max():.3e} rms {np.sqrt(np.mean(d * d)):.3e}", flush=True)


CASES = [
    (1.0, 30.0, (40, 70), 1),      # W = 3, one tile wide, ragged
    (3.0, 30.0, (96, 130), 2),     # W = 9: 2 x 3 tiles
    (3.0, 10.0, (64, 64), 3),      # exactly one tile, high order
    (5.0, 40.0, (129, 65), 4),     # one-pixel tails
    (10.0, 50.0, (150, 170), 5),   # W = 30
    (15.0, 30.0, (140, 133), 6),   # W = 45, the widest the tile holds
    (2.0, 12.0, (66, 67), 7),      # small sigma_r
    (0.3, 25.0, (70, 90), 8),      # W = 1
]


@pytest.mark.parametrize("ss,sr,shape,seed", CASES)
def test_matches_alg2(ss, sr, shape, seed):
    f = synthimg.gen2(*shape, seed)
    out, plan, f32 = _forward(f, sr, ss)
    ref = G.gpa_alg2(f32, K.taps1d("gauss", ss), sr, plan.info.N, 127.5)
    print(f"sigma_s={ss} sr={sr} {shape}: N={plan.info.N} W={plan.info.W}", flush=True)
    _report("gpu-alg2", out - ref)
    assert np.abs(out - ref).max() <= TOL


@pytest.mark.parametrize("shape", [(1, 1), (1, 200), (200, 1), (3, 3), (5, 64), (64, 5), (65, 129)])
def test_ragged_and_tiny(shape):
    f = synthimg.gen1(*shape, 31)
    out, plan, f32 = _forward(f, 25.0, 2.0)
    ref = G.gpa_alg2(f32, K.taps1d("gauss", 2.0), 25.0, plan.info.N, 127.5)
    assert np.abs(out - ref).max() <= TOL, shape


def test_image_narrower_than_halo():
    # W = 36 on a 20 x 30 image: every region slot but the image is padding
    f = synthimg.gen2(20, 30, 32)
    out, plan, f32 = _forward(f, 30.0, 12.0)
    ref = G.gpa_alg2(f32, K.taps1d("gauss", 12.0), 30.0, plan.info.N, 127.5)
    assert np.abs(out - ref).max() <= TOL


def test_workload1_vs_oracles():
    # 256^2 gen1, sigma_s = 3 (W = 9), sigma_r = 30, N from delta = 1e-3
    f = synthimg.gen1(256, 256, 1000)
    out, plan, f32 = _forward(f, 30.0, 3.0)
    assert plan.info.N == 48 and plan.info.W == 9
    o3 = G.gpa_alg2(f32, K.taps1d("gauss", 3.0), 30.0, 48, 127.5)
    o1 = B.direct_bf(f32, K.taps2d("gauss", 3.0), 30.0)
    _report("gpu-O3", out - o3)
    _report("gpu-O1", out - o1)
    assert np.abs(out - o3).max() <= TOL
    assert np.abs(out - o1).max() <= TOL


@pytest.mark.parametrize("ss,sr", [(3.0, 10.0), (10.0, 30.0)])
def test_full_size_sampled(ss, sr):
    # 4096^2 gen2 in the launch configuration of the timed sweep, checked
    # pixel by pixel on a sample (borders, corners, tile seams, interior)
    f = synthimg.gen2(4096, 4096, 4000)
    out, plan, f32 = _forward(f, sr, ss)
    W = plan.info.W
    px = synthimg.sample_pixels(4096, 4096, 600, W, 200, 4001)
    o2 = G.gpa_pairwise_at(f32, px, K.taps2d("gauss", ss), sr, plan.info.N, 127.5)
    got = out[px[:, 0], px[:, 1]]
    print(f"N={plan.info.N} W={W} pixels={len(px)}", flush=True)
    _report("gpu-O2", got - o2)
    assert np.abs(got - o2).max() <= TOL


@pytest.mark.parametrize("ss,sr,shape", [(2.0, 30.0, (45, 71)), (4.0, 20.0, (100, 90)), (15.0, 40.0, (70, 60))])
def test_mirror_matches_oracle(ss, sr, shape):
    f = synthimg.gen2(*shape, 61)
    out, plan, f32 = _forward(f, sr, ss, mirror=True)
    ref = M.gpa_alg2(f32, K.taps1d("gauss", ss), sr, plan.info.N, 127.5)
    _report("gpu-mirror", out - ref)
    assert np.abs(out - ref).max() <= TOL


def test_agrees_with_valu_tile():
    torch, P = _mods()
    f = synthimg.gen2(300, 257, 71)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    a = P.Plan("gauss", 20.0, 300, 257, sigma_s=4.0, engine="mfma").forward(x)
    b = P.Plan("gauss", 20.0, 300, 257, sigma_s=4.0, engine="valu").forward(x)
    torch.cuda.synchronize()
    assert (a - b).abs().max().item() <= TOL


@pytest.mark.parametrize("ss,sr,shape,seed,use_saved", [(2.0, 30.0, (45, 71), 3, True),
                                                        (3.0, 25.0, (66, 90), 4, False)])
def test_adjoint_from_mfma_state(ss, sr, shape, seed, use_saved):
    # the saved planes (Q, ratio, D_c) written by this engine feed bf_backward
    torch, P = _mods()
    f = synthimg.gen1(*shape, seed)
    gbar = synthimg.gen2(*shape, seed + 100) / 255.0 - 0.5
    H, Wd = shape
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    g = torch.tensor(gbar, dtype=torch.float32, device="cuda")
    plan = P.Plan("gauss", sr, H, Wd, sigma_s=ss, grad=True, engine="mfma")
    assert plan.info.path == P.BF_PATH_TILE_MFMA
    saved = plan.new_saved() if use_saved else None
    plan.forward(x, saved=saved)
    gin, gs = plan.backward(x, g, saved=saved)
    torch.cuda.synchronize()
    f32 = x.cpu().numpy().astype(np.float64)
    g32 = g.cpu().numpy().astype(np.float64)
    df, dsr, dss = GR.vjp_autograd(f32, g32, "gauss", ss, plan.info.W, sr, plan.info.N, 127.5)
    gin = gin.cpu().numpy().astype(np.float64)
    gs = gs.cpu().numpy()
    err = np.abs(gin - df).max() / np.abs(df).max()
    print(f"df rel {err:.2e} dsr {gs[0]:.6e} vs {dsr:.6e} dss {gs[1]:.6e} vs {dss:.6e}", flush=True)
    assert err <= RTOL
    assert abs(gs[0] - dsr) <= RTOL * abs(dsr)
    assert abs(gs[1] - dss) <= RTOL * abs(dss)
