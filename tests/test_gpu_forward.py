"""GPU parity of the fused forward (bf_forward) against the FP64 CPU oracle.

Tolerance: max |GPU - oracle| <= 1e-3 on the 0-255 intensity scale (the
accuracy target of the workloads), with the oracle evaluated in float64 on
the float32-rounded input the GPU sees and at the same order N.
"""
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


def _taps(kind, kw):
    return K.taps1d(kind, kw.get("sigma_s"), kw.get("W") if kind == "box" else None), \
        K.taps2d(kind, kw.get("sigma_s"), kw.get("W") if kind == "box" else None)


def _gpu_forward(f, kind, sr, **kw):
    torch, P = _mods()
    H, Wd = f.shape
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    plan = P.Plan(kind, sr, H, Wd, **kw)
    out = plan.forward(x)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), plan, x.cpu().numpy().astype(np.float64)


def _report(name, d):
    print(f"{name}: max {np.abs(d).max():.3e} rms {np.sqrt(np.mean(d * d)):.3e}", flush=True)


CASES = [
    ("box", dict(W=1), 30.0, (37, 45), 1),
    ("box", dict(W=5), 20.0, (150, 133), 2),
    ("box", dict(W=10), 30.0, (100, 200), 3),
    ("box", dict(W=30), 30.0, (130, 150), 4),
    ("box", dict(W=5), 10.0, (70, 80), 5),
    ("gauss", dict(sigma_s=1.0), 30.0, (40, 70), 6),
    ("gauss", dict(sigma_s=3.0), 30.0, (96, 130), 7),
    ("gauss", dict(sigma_s=5.0), 40.0, (80, 100), 8),
    ("gauss", dict(sigma_s=10.0), 50.0, (90, 90), 9),
    ("gauss", dict(sigma_s=2.0), 12.0, (66, 67), 10),
]


@pytest.mark.parametrize("kind,kw,sr,shape,seed", CASES)
def test_forward_matches_alg2(kind, kw, sr, shape, seed):
    f = synthimg.gen2(*shape, seed)
    out, plan, f32 = _gpu_forward(f, kind, sr, **kw)
    w1, _ = _taps(kind, kw)
    ref = G.gpa_alg2(f32, w1, sr, plan.info.N, 127.5)
    print(f"{kind} {kw} sr={sr} {shape}: N={plan.info.N} tile={plan.info.tile_rows}", flush=True)
    _report("gpu-alg2", out - ref)
    assert np.abs(out - ref).max() <= TOL


@pytest.mark.parametrize("fp32", [False, True])
def test_workload1_vs_oracles(fp32):
    # 256^2 gen1, Gaussian sigma_s = 3 (W = 9), sigma_r = 30, N from delta = 1e-3
    f = synthimg.gen1(256, 256, 1000)
    out, plan, f32 = _gpu_forward(f, "gauss", 30.0, sigma_s=3.0, fp32_accum=fp32)
    assert plan.info.N == 48 and plan.info.W == 9
    w1, w2 = K.taps1d("gauss", 3.0), K.taps2d("gauss", 3.0)
    o3 = G.gpa_alg2(f32, w1, 30.0, 48, 127.5)
    o1 = B.direct_bf(f32, w2, 30.0)
    _report("gpu-O3", out - o3)
    _report("gpu-O1", out - o1)
    assert np.abs(out - o3).max() <= TOL
    assert np.abs(out - o1).max() <= TOL


@pytest.mark.parametrize("kind,kw,sr", [("box", dict(W=5), 20.0), ("box", dict(W=5), 40.0),
                                        ("gauss", dict(sigma_s=5.0), 20.0),
                                        ("gauss", dict(sigma_s=5.0), 40.0)])
def test_workload2_sampled(kind, kw, sr):
    # 1024^2 gen2 (blocks + ramp + noise): checked pixel by pixel on a sample
    f = synthimg.gen2(1024, 1024, 2000)
    out, plan, f32 = _gpu_forward(f, kind, sr, **kw)
    _, w2 = _taps(kind, kw)
    W = plan.info.W
    px = synthimg.sample_pixels(1024, 1024, 1500, W, 500, 2001)
    o2 = G.gpa_pairwise_at(f32, px, w2, sr, plan.info.N, 127.5)
    o1 = B.direct_bf_at(f32, px, w2, sr)
    got = out[px[:, 0], px[:, 1]]
    print(f"N={plan.info.N} pixels={len(px)}", flush=True)
    _report("gpu-O2", got - o2)
    _report("gpu-O1", got - o1)
    assert np.abs(got - o2).max() <= TOL
    assert np.abs(got - o1).max() <= TOL


@pytest.mark.parametrize("shape", [(1, 1), (1, 200), (200, 1), (3, 3), (5, 64), (64, 5), (65, 129)])
def test_ragged_and_tiny(shape):
    f = synthimg.gen1(*shape, 31)
    for kind, kw in [("box", dict(W=3)), ("gauss", dict(sigma_s=2.0))]:
        out, plan, f32 = _gpu_forward(f, kind, 25.0, **kw)
        w1, _ = _taps(kind, kw)
        ref = G.gpa_alg2(f32, w1, 25.0, plan.info.N, 127.5)
        assert np.abs(out - ref).max() <= TOL, (kind, shape)


@pytest.mark.parametrize("shape", [(1, 1), (1, 200), (200, 1), (3, 3), (5, 64), (64, 5), (65, 129)])
def test_ragged_and_tiny_wide_gaussian(shape):
    # Gaussians from W = 16 on take the streamed passes at every image size: W = 18 (matrix-core
    # column pass) and W = 45 (split column pass), supports far beyond the image
    f = synthimg.gen1(*shape, 33)
    for ss in (6.0, 15.0):
        out, plan, f32 = _gpu_forward(f, "gauss", 25.0, sigma_s=ss)
        assert plan.info.path == 1, (ss, shape)  # streamed
        w1, _ = _taps("gauss", dict(sigma_s=ss))
        ref = G.gpa_alg2(f32, w1, 25.0, plan.info.N, 127.5)
        assert np.abs(out - ref).max() <= TOL, (ss, shape)


def test_support_zero_is_identity():
    f = synthimg.gen2(50, 70, 41)
    out, plan, f32 = _gpu_forward(f, "box", 30.0, W=0)
    assert np.abs(out - f32).max() <= TOL


def test_constant_image():
    f = np.full((77, 91), 203.5)
    for kind, kw in [("box", dict(W=7)), ("gauss", dict(sigma_s=4.0))]:
        out, plan, _ = _gpu_forward(f, kind, 30.0, **kw)
        assert np.abs(out - 203.5).max() <= TOL


def test_pitched_buffers():
    torch, P = _mods()
    f = synthimg.gen2(90, 100, 51)
    big_in = torch.zeros(90, 128, dtype=torch.float32, device="cuda")
    big_in[:, :100] = torch.tensor(f, dtype=torch.float32, device="cuda")
    big_out = torch.full((90, 160), -7.0, dtype=torch.float32, device="cuda")
    plan = P.Plan("gauss", 30.0, 90, 100, sigma_s=2.5)
    plan.forward(big_in[:, :100], out=big_out[:, :100])
    torch.cuda.synchronize()
    o = big_out.cpu().numpy().astype(np.float64)
    ref = G.gpa_alg2(big_in[:, :100].cpu().numpy().astype(np.float64), K.taps1d("gauss", 2.5), 30.0,
                     plan.info.N, 127.5)
    assert np.abs(o[:, :100] - ref).max() <= TOL
    assert np.all(o[:, 100:] == -7.0)  # nothing written past the width


def test_deterministic():
    torch, P = _mods()
    f = synthimg.gen2(300, 257, 61)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    plan = P.Plan("box", 30.0, 300, 257, W=9)
    a = plan.forward(x).clone()
    b = plan.forward(x)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_explicit_order_and_rules():
    torch, P = _mods()
    f = synthimg.gen1(60, 60, 71)
    out, plan, f32 = _gpu_forward(f, "box", 30.0, W=4, N=20)
    assert plan.info.N == 20 and plan.info.status == 1  # BF_WNOGUARANTEE
    ref = G.gpa_alg2(f32, K.taps1d("box", W=4), 30.0, 20, 127.5)
    assert np.abs(out - ref).max() <= TOL


# --- large supports: the blocked path through device memory ---------------

@pytest.mark.parametrize("kind,kw,sr,shape", [("box", dict(W=75), 50.0, (200, 330)),
                                              ("box", dict(W=75), 10.0, (90, 170)),
                                              ("gauss", dict(sigma_s=25.0), 30.0, (170, 260)),
                                              ("gauss", dict(sigma_s=16.0, streamed=True), 12.0, (100, 140)),
                                              ("box", dict(W=60), 30.0, (40, 50))])
def test_large_support(kind, kw, sr, shape):
    f = synthimg.gen2(*shape, 77)
    out, plan, f32 = _gpu_forward(f, kind, sr, **kw)
    assert plan.info.path == 1  # streamed path
    kw = {k: v for k, v in kw.items() if k != "streamed"}
    w1, _ = _taps(kind, kw)
    ref = G.gpa_alg2(f32, w1, sr, plan.info.N, 127.5)
    print(f"{kind} {kw} sr={sr} N={plan.info.N}", flush=True)
    _report("gpu-alg2", out - ref)
    assert np.abs(out - ref).max() <= TOL


@pytest.mark.parametrize("kind,kw,sr", [("box", dict(W=7), 30.0), ("gauss", dict(sigma_s=3.0), 20.0)])
def test_streamed_matches_fused(kind, kw, sr):
    torch, P = _mods()
    f = synthimg.gen2(150, 210, 78)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    a = P.Plan(kind, sr, 150, 210, **kw).forward(x)
    ps = P.Plan(kind, sr, 150, 210, streamed=True, **kw)
    b = ps.forward(x)
    torch.cuda.synchronize()
    assert ps.info.path == 1
    assert (a - b).abs().max().item() <= 1e-4
    w1, _ = _taps(kind, kw)
    ref = G.gpa_alg2(x.cpu().numpy().astype(np.float64), w1, sr, ps.info.N, 127.5)
    assert np.abs(b.cpu().numpy() - ref).max() <= TOL


@pytest.mark.parametrize("kind,kw,sr", [("box", dict(W=75), 30.0), ("gauss", dict(sigma_s=25.0), 50.0),
                                        ("box", dict(W=30), 10.0), ("gauss", dict(sigma_s=10.0), 30.0)])
def test_workload3_sampled(kind, kw, sr):
    # 4096^2 gen2, checked pixel by pixel on a sample (incl. the border band)
    f = synthimg.gen2(4096, 4096, 3000)
    out, plan, f32 = _gpu_forward(f, kind, sr, **kw)
    _, w2 = _taps(kind, kw)
    W = plan.info.W
    n = 60 if W > 40 else 300
    px = synthimg.sample_pixels(4096, 4096, n, W, n // 3, 3001)
    o2 = G.gpa_pairwise_at(f32, px, w2, sr, plan.info.N, 127.5)
    got = out[px[:, 0], px[:, 1]]
    print(f"N={plan.info.N} pixels={len(px)} tile_rows={plan.info.tile_rows}", flush=True)
    _report("gpu-O2", got - o2)
    assert np.abs(got - o2).max() <= TOL


@pytest.mark.parametrize("kind,kw,sr", [("box", dict(W=6), 25.0), ("gauss", dict(sigma_s=3.0), 30.0)])
def test_streamed_saved_state_matches_fused(kind, kw, sr):
    # the forward's saved planes (for the adjoint) agree between the two paths
    torch, P = _mods()
    f = synthimg.gen2(140, 200, 79)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    pf = P.Plan(kind, sr, 140, 200, grad=True, **kw)
    ps = P.Plan(kind, sr, 140, 200, grad=True, streamed=True, **kw)
    assert ps.info.path == 1 and pf.info.path == 0
    sf, ss = pf.new_saved(), ps.new_saved()
    a = pf.forward(x, saved=sf)
    b = ps.forward(x, saved=ss)
    torch.cuda.synchronize()
    assert (a - b).abs().max().item() <= 1e-4
    for i, (u, v) in enumerate(zip(sf.view(3, -1), ss.view(3, -1))):
        scale = u.abs().max().item()
        assert (u - v).abs().max().item() <= 1e-4 * scale + 1e-12, i


def test_clone_workspace_on_two_streams():
    # a clone has its own workspace: both plans run at once on two streams
    torch, P = _mods()
    f = synthimg.gen2(300, 280, 81)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    for kind, kw in [("gauss", dict(sigma_s=25.0)), ("box", dict(W=5))]:
        a = P.Plan(kind, 20.0, 300, 280, **kw)
        b = a.clone()
        assert b.info.N == a.info.N and b.info.W == a.info.W and b.info.tile_rows == a.info.tile_rows
        ref = a.forward(x)
        torch.cuda.synchronize()
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        o1, o2 = torch.empty_like(x), torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            a.forward(x, out=o1, stream=s1)
            b.forward(x, out=o2, stream=s2)
        torch.cuda.synchronize()
        assert torch.equal(o1, ref) and torch.equal(o2, ref)


@pytest.mark.parametrize("W,sr,shape", [(16, 10.0, (150, 700)), (56, 30.0, (120, 1100)), (75, 20.0, (90, 900)),
                                        (190, 30.0, (60, 500)), (20, 15.0, (140, 900)), (40, 25.0, (100, 1300))])
def test_box_strip_widths_agree(W, sr, shape):
    # the forward-only strips (512 columns from W = 48) against the
    # 256-column strips that also write the saved state, and both against the
    # oracle; several strips, a ragged last one.  W = 20 (N = 133) and W = 40
    # (N = 66) end their 32-order launches with a 16-order one.
    torch, P = _mods()
    f = synthimg.gen2(*shape, 80 + W)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    pa = P.Plan("box", sr, *shape, W=W, engine="streamed")
    a = pa.forward(x)
    ref = G.gpa_alg2(x.cpu().numpy().astype(np.float64), K.taps1d("box", W=W), sr, pa.info.N, 127.5)
    da = np.abs(a.cpu().numpy() - ref).max()
    db = 0.0
    if W <= 120:  # the adjoint's support limit: only then is there a saved-state plan
        pg = P.Plan("box", sr, *shape, W=W, engine="streamed", grad=True)
        b = pg.forward(x, saved=pg.new_saved())
        torch.cuda.synchronize()
        db = np.abs(b.cpu().numpy() - ref).max()
    print(f"W={W} N={pa.info.N}: wide {da:.3e} saved {db:.3e}", flush=True)
    assert da <= TOL and db <= TOL
