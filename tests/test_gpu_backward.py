"""GPU parity of the adjoint (bf_backward) against float64 CPU gradients.

References: oracle.grad.vjp_autograd (float64 torch autograd through
Algorithm 2) on the float32-rounded input the GPU sees, and central finite
differences (h = 1e-3) of the numpy Algorithm 2 at sampled pixels.
Tolerance: max |GPU - ref| <= 1e-3 * max |ref| for dL/df, and relative
1e-3 for the two sigma gradients.
"""
import numpy as np
import pytest

import synthimg
from oracle import gpa as G
from oracle import grad as GR
from oracle import kernels as K

pytestmark = pytest.mark.gpu
RTOL = 1e-3


def _mods():
    import torch
    import paper_1603_08109_amd as P
    assert torch.cuda.is_available()
    return torch, P


def _run(f, gbar, kind, sr, use_saved=True, **kw):
    torch, P = _mods()
    H, Wd = f.shape
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    g = torch.tensor(gbar, dtype=torch.float32, device="cuda")
    plan = P.Plan(kind, sr, H, Wd, grad=True, **kw)
    saved = plan.new_saved() if use_saved else None
    plan.forward(x, saved=saved)
    gin, gs = plan.backward(x, g, saved=saved)
    torch.cuda.synchronize()
    return (gin.cpu().numpy().astype(np.float64), gs.cpu().numpy(), plan,
            x.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64))


CASES = [
    ("box", dict(W=3), 30.0, (40, 50), 1),
    ("box", dict(W=8), 20.0, (70, 83), 2),
    ("gauss", dict(sigma_s=2.0), 30.0, (45, 71), 3),
    ("gauss", dict(sigma_s=3.0), 25.0, (66, 90), 4),
    ("gauss", dict(sigma_s=5.0), 30.0, (64, 64), 5),
]


@pytest.mark.parametrize("kind,kw,sr,shape,seed", CASES)
def test_adjoint_matches_autograd(kind, kw, sr, shape, seed):
    f = synthimg.gen1(*shape, seed)
    gbar = synthimg.gen2(*shape, seed + 100) / 255.0 - 0.5
    gin, gs, plan, f32, g32 = _run(f, gbar, kind, sr, **kw)
    W = plan.info.W
    df, dsr, dss = GR.vjp_autograd(f32, g32, kind, kw.get("sigma_s"), W, sr, plan.info.N, 127.5)
    err = np.abs(gin - df).max() / np.abs(df).max()
    print(f"{kind} {kw} N={plan.info.N}: df rel {err:.2e}  dsr {gs[0]:.6e} vs {dsr:.6e}  "
          f"dss {gs[1]:.6e} vs {dss:.6e}", flush=True)
    assert err <= RTOL
    assert abs(gs[0] - dsr) <= RTOL * abs(dsr)
    if kind == "gauss":
        assert abs(gs[1] - dss) <= RTOL * abs(dss)
    else:
        assert np.isnan(gs[1])


def test_recompute_equals_saved():
    f = synthimg.gen1(50, 77, 7)
    gbar = synthimg.gen2(50, 77, 8) / 255.0 - 0.5
    a = _run(f, gbar, "gauss", 30.0, True, sigma_s=2.0)
    b = _run(f, gbar, "gauss", 30.0, False, sigma_s=2.0)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])


def test_adjoint_vs_finite_differences():
    # central differences (h = 1e-3) of the float64 numpy Algorithm 2
    f = synthimg.gen1(24, 30, 9)
    target = synthimg.clean_blocks(24, 30, 9)
    kind, ss, sr = "gauss", 1.5, 30.0
    torch, P = _mods()
    plan = P.Plan(kind, sr, 24, 30, sigma_s=ss, grad=True)
    f32 = np.asarray(f, np.float32).astype(np.float64)
    out = G.gpa_alg2(f32, K.taps1d(kind, ss), sr, plan.info.N, 127.5)
    gbar = 2.0 * (out - target) / out.size
    gin, gs, plan, f32, g32 = _run(f32, gbar, kind, sr, sigma_s=ss)
    px = np.array([[0, 0], [5, 7], [12, 29], [23, 14], [17, 3]])
    fd, fdsr, fdss = GR.vjp_fd(f32, g32, kind, ss, plan.info.W, sr, plan.info.N, 127.5, px)
    scale = np.abs(gin).max()
    assert np.abs(gin[px[:, 0], px[:, 1]] - fd).max() <= RTOL * scale
    assert abs(gs[0] - fdsr) <= RTOL * abs(fdsr)
    assert abs(gs[1] - fdss) <= RTOL * abs(fdss)


def test_workload5_one_image():
    # 512^2 gen1, Gaussian sigma_s = 5, sigma_r = 30, N = 49, MSE loss vs clean blocks
    torch, P = _mods()
    f = synthimg.gen1(512, 512, 5000)
    target = synthimg.clean_blocks(512, 512, 5000)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    plan = P.Plan("gauss", 30.0, 512, 512, sigma_s=5.0, grad=True)
    assert plan.info.N == 49
    saved = plan.new_saved()
    out = plan.forward(x, saved=saved)
    gbar = 2.0 * (out.double() - torch.tensor(target, device="cuda")) / out.numel()
    g32 = gbar.float()
    gin, gs = plan.backward(x, g32, saved=saved)
    torch.cuda.synchronize()
    f32 = x.cpu().numpy().astype(np.float64)
    df, dsr, dss = GR.vjp_autograd(f32, g32.cpu().numpy().astype(np.float64), "gauss", 5.0, 15, 30.0,
                                   49, 127.5)
    gi = gin.cpu().numpy()
    err = np.abs(gi - df).max() / np.abs(df).max()
    print(f"df rel {err:.2e} rms {np.sqrt(np.mean((gi - df) ** 2)) / np.abs(df).max():.2e} "
          f"dsr {gs[0].item():.6e}/{dsr:.6e} dss {gs[1].item():.6e}/{dss:.6e}", flush=True)
    assert err <= RTOL
    assert abs(gs[0].item() - dsr) <= RTOL * abs(dsr)
    assert abs(gs[1].item() - dss) <= RTOL * abs(dss)


def test_autograd_module():
    torch, P = _mods()
    f = synthimg.gen1(48, 64, 13)
    target = torch.tensor(synthimg.clean_blocks(48, 64, 13), dtype=torch.float32, device="cuda")
    x = torch.tensor(f, dtype=torch.float32, device="cuda", requires_grad=True)
    m = P.BilateralGPA("gauss", sigma_r=30.0, sigma_s=2.0).cuda()
    y = m(x)
    loss = ((y - target) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    f32 = f.astype(np.float32).astype(np.float64)
    out = G.gpa_alg2(f32, K.taps1d("gauss", 2.0), 30.0, m._N, 127.5)
    gbar = 2.0 * (y.detach().double().cpu().numpy() - target.cpu().numpy()) / y.numel()
    df, dsr, dss = GR.vjp_autograd(f32, gbar, "gauss", 2.0, m.W, 30.0, m._N, 127.5)
    assert np.abs(y.detach().cpu().numpy() - out).max() <= 1e-3
    assert np.abs(x.grad.cpu().numpy() - df).max() <= RTOL * np.abs(df).max()
    assert abs(m.sigma_r.grad.item() - dsr) <= RTOL * abs(dsr)
    assert abs(m.sigma_s.grad.item() - dss) <= RTOL * abs(dss)


# --- streamed adjoint (supports wider than the fused adjoint tiles) --------

@pytest.mark.parametrize("kind,kw,sr,shape,seed", [
    ("gauss", dict(sigma_s=12.0), 30.0, (60, 90), 11),   # W = 36: streamed adjoint by size
    ("box", dict(W=40), 25.0, (70, 100), 12),
    ("gauss", dict(sigma_s=2.0, streamed=True), 30.0, (45, 71), 13),
    ("box", dict(W=4, streamed=True), 20.0, (50, 66), 14),
])
def test_streamed_adjoint_matches_autograd(kind, kw, sr, shape, seed):
    f = synthimg.gen1(*shape, seed)
    gbar = synthimg.gen2(*shape, seed + 100) / 255.0 - 0.5
    for use_saved in (True, False):
        gin, gs, plan, f32, g32 = _run(f, gbar, kind, sr, use_saved=use_saved, **kw)
        W = plan.info.W
        df, dsr, dss = GR.vjp_autograd(f32, g32, kind, kw.get("sigma_s"), W, sr, plan.info.N, 127.5)
        err = np.abs(gin - df).max() / np.abs(df).max()
        print(f"{kind} {kw} saved={use_saved} N={plan.info.N}: df rel {err:.2e}  dsr {gs[0]:.6e} vs "
              f"{dsr:.6e}  dss {gs[1]:.6e} vs {dss:.6e}", flush=True)
        assert err <= RTOL
        assert abs(gs[0] - dsr) <= RTOL * abs(dsr)
        if kind == "gauss":
            assert abs(gs[1] - dss) <= RTOL * abs(dss)
        else:
            assert np.isnan(gs[1])


@pytest.mark.parametrize("kind,kw,sr", [("box", dict(W=6), 30.0), ("gauss", dict(sigma_s=3.0), 20.0)])
def test_streamed_adjoint_matches_fused(kind, kw, sr):
    torch, P = _mods()
    f = synthimg.gen2(130, 190, 15)
    gbar = synthimg.gen1(130, 190, 16) / 255.0 - 0.5
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    g = torch.tensor(gbar, dtype=torch.float32, device="cuda")
    res = []
    for streamed in (False, True):
        plan = P.Plan(kind, sr, 130, 190, grad=True, streamed=streamed, **kw)
        gin, gs = plan.backward(x, g)  # recomputes the forward state
        torch.cuda.synchronize()
        res.append((gin.cpu().numpy().astype(np.float64), gs.cpu().numpy()))
    (a, sa), (b, sb) = res
    # both compute the filters in float32 in different summation orders (VALU
    # tiles vs matrix-core Toeplitz blocks); the float64 reference decides
    W = P.Plan(kind, sr, 130, 190, **kw).info.W
    N = P.Plan(kind, sr, 130, 190, **kw).info.N
    df, dsr, dss = GR.vjp_autograd(x.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64),
                                   kind, kw.get("sigma_s"), W, sr, N, 127.5)
    print(f"dsr fused {sa[0]:.9e} streamed {sb[0]:.9e} fp64 {dsr:.9e}; "
          f"dss fused {sa[1]:.9e} streamed {sb[1]:.9e} fp64 {dss:.9e}", flush=True)
    assert np.abs(a - b).max() <= 1e-4 * np.abs(a).max()
    assert abs(sa[0] - sb[0]) <= 1e-4 * abs(dsr)
    assert abs(sb[0] - dsr) <= RTOL * abs(dsr)
    if kind == "gauss":
        assert abs(sa[1] - sb[1]) <= 1e-4 * abs(dss)
        assert abs(sb[1] - dss) <= RTOL * abs(dss)
