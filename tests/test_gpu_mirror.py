"""GPU parity of the reflecting (mirror) border, BF_FLAG_MIRROR, against the
float64 oracle (oracle.mirror): fused tiles (including supports wider than
the image, i.e. repeated reflections), the streamed paths (box strips and the
matrix-core Gaussian), a sampled 4096^2 check, the batch, the cross filter,
and the unsupported combinations.  Tolerance 1e-3 on the 0-255 scale."""
import numpy as np
import pytest

import synthimg
from oracle import joint as J
from oracle import kernels as K
from oracle import mirror as M

pytestmark = pytest.mark.gpu
TOL = 1e-3


def _mods():
    import torch
    import paper_1603_08109_amd as P
    assert torch.cuda.is_available()
    return torch, P


def _w1(kind, kw):
    return K.taps1d(kind, kw.get("sigma_s"), kw.get("W") if kind == "box" else None)


def _run(f, kind, sr, **kw):
    torch, P = _mods()
    H, Wd = f.shape
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    plan = P.Plan(kind, sr, H, Wd, mirror=True, **kw)
    out = plan.forward(x)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), plan, x.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("kind,kw,sr,shape", [("box", dict(W=3), 30.0, (40, 55)), ("box", dict(W=9), 20.0, (5, 7)),
                                              ("gauss", dict(sigma_s=2.0), 25.0, (70, 64)),
                                              ("gauss", dict(sigma_s=3.0), 40.0, (9, 130)),
                                              ("gauss", dict(sigma_s=1.0), 15.0, (1, 1))])
def test_fused_mirror(kind, kw, sr, shape):
    f = synthimg.gen2(*shape, 61)
    out, plan, f32 = _run(f, kind, sr, **kw)
    assert plan.info.path == 0
    ref = M.gpa_alg2(f32, _w1(kind, kw), sr, plan.info.N, 127.5)
    print(f"{kind} {kw} {shape}: max {np.abs(out - ref).max():.3e}", flush=True)
    assert np.abs(out - ref).max() <= TOL


@pytest.mark.parametrize("kind,kw,sr,shape", [("box", dict(W=20), 30.0, (90, 150)), ("box", dict(W=60), 20.0, (70, 50)),
                                              ("gauss", dict(sigma_s=5.0), 25.0, (100, 120)),
                                              ("gauss", dict(sigma_s=12.0), 35.0, (60, 90))])
def test_streamed_mirror(kind, kw, sr, shape):
    f = synthimg.gen2(*shape, 62)
    out, plan, f32 = _run(f, kind, sr, streamed=True, **kw)
    assert plan.info.path == 1
    ref = M.gpa_alg2(f32, _w1(kind, kw), sr, plan.info.N, 127.5)
    print(f"{kind} {kw} {shape}: max {np.abs(out - ref).max():.3e}", flush=True)
    assert np.abs(out - ref).max() <= TOL


@pytest.mark.parametrize("kind,kw,sr", [("box", dict(W=75), 30.0), ("gauss", dict(sigma_s=25.0), 50.0)])
def test_mirror_workload_sampled(kind, kw, sr):
    f = synthimg.gen2(4096, 4096, 3000)
    out, plan, f32 = _run(f, kind, sr, **kw)
    w2 = K.taps2d(kind, kw.get("sigma_s"), kw.get("W") if kind == "box" else None)
    px = synthimg.sample_pixels(4096, 4096, 40, plan.info.W, 40, 3002)
    got = out[px[:, 0], px[:, 1]]
    ref = M.gpa_pairwise_at(f32, px, w2, sr, plan.info.N, 127.5)
    print(f"N={plan.info.N} tile_rows={plan.info.tile_rows}: max {np.abs(got - ref).max():.3e}", flush=True)
    assert np.abs(got - ref).max() <= TOL


def test_batch_mirror_equals_plans():
    torch, P = _mods()
    specs = [dict(kernel="box", W=4, sigma_r=30.0, height=50, width=61, mirror=True),
             dict(kernel="gauss", sigma_s=2.5, sigma_r=20.0, height=33, width=90, mirror=True),
             dict(kernel="gauss", sigma_s=1.5, sigma_r=40.0, height=70, width=40)]
    batch = P.Batch(specs)
    imgs = [torch.tensor(synthimg.gen2(s["height"], s["width"], 63 + i), dtype=torch.float32, device="cuda")
            for i, s in enumerate(specs)]
    outs = batch.forward(imgs)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        kw = {k: v for k, v in s.items() if k not in ("kernel", "sigma_r", "height", "width")}
        ref = P.Plan(s["kernel"], s["sigma_r"], s["height"], s["width"], **kw).forward(imgs[i])
        torch.cuda.synchronize()
        assert (outs[i] - ref).abs().max().item() <= 1e-4, i


def test_joint_mirror():
    torch, P = _mods()
    f = synthimg.gen2(40, 52, 64)
    h = synthimg.gen1(40, 52, 65)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    g = torch.tensor(h, dtype=torch.float32, device="cuda")
    plan = P.Plan("gauss", 25.0, 40, 52, sigma_s=2.0, joint=True, mirror=True)
    out = plan.forward_joint(x, g).cpu().numpy().astype(np.float64)
    W = plan.info.W
    fp = np.pad(x.cpu().numpy().astype(np.float64), W, mode="symmetric")
    hp = np.pad(g.cpu().numpy().astype(np.float64), W, mode="symmetric")
    ref = J.gpa_joint_alg2(fp, hp, K.taps1d("gauss", 2.0), 25.0, plan.info.N, 127.5)[W:W + 40, W:W + 52]
    assert np.abs(out - ref).max() <= TOL


def test_mirror_unsupported():
    torch, P = _mods()
    with pytest.raises(P.BFError):
        P.Plan("box", 30.0, 300, 300, W=120, mirror=True)  # streamed box beyond the strips
