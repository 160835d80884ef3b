"""GPU parity of the video/volume path (bf_plan_volume / bf_forward_volume)
against the FP64 oracle twin ``oracle.volume``.

Tolerance: max |GPU - oracle| <= 1e-3 on the 0-255 scale, oracle in float64
on the float32-rounded input at the same N.  Shapes cover one slice (which
must equal the 2-D filter), fewer slices than the support, ragged tiles in
every axis, a 64-frame 256^2 video at sampled voxels, and the mirror border
(also with fewer slices and slice rows than the support)."""
import numpy as np
import pytest

import synthimg
from oracle import gpa as G
from oracle import kernels as K
from oracle import volume as V

pytestmark = pytest.mark.gpu
TOL = 1e-3


def _mods():
    import torch
    import paper_1603_08109_amd as P
    assert torch.cuda.is_available()
    return torch, P


def _vol(D, H, W, seed):
    return np.stack([synthimg.gen2(H, W, seed + 7 * d) for d in range(D)])


def _run(f, kind, sr, **kw):
    torch, P = _mods()
    D, H, Wd = f.shape
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    plan = P.VolumePlan(kind, sr, D, H, Wd, **kw)
    assert plan.info.path == P.BF_PATH_VOLUME
    out = plan.forward(x)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), plan, x.cpu().numpy().astype(np.float64)


def _w1(kind, kw):
    return K.taps1d(kind, kw.get("sigma_s"), kw.get("W") if kind == "box" else None)


CASES = [
    ("box", dict(W=2), 30.0, (5, 37, 45), 1),
    ("gauss", dict(sigma_s=1.5), 30.0, (8, 64, 70), 2),
    ("box", dict(W=7), 20.0, (3, 20, 300), 3),
    ("gauss", dict(sigma_s=2.0), 10.0, (17, 33, 17), 4),
    ("box", dict(W=5), 40.0, (2, 30, 40), 5),     # fewer slices than the support
    ("gauss", dict(sigma_s=1.0), 50.0, (9, 130, 65), 6),
]


@pytest.mark.parametrize("kind,kw,sr,shape,seed", CASES)
def test_matches_oracle(kind, kw, sr, shape, seed):
    f = _vol(*shape, seed)
    out, plan, f32 = _run(f, kind, sr, **kw)
    ref = V.gpa_alg2(f32, _w1(kind, kw), sr, plan.info.N, 127.5)
    d = np.abs(out - ref)
    print(f"{kind} {kw} sr={sr} {shape}: N={plan.info.N} max {d.max():.3e}", flush=True)
    assert d.max() <= TOL


@pytest.mark.parametrize("kind,kw", [("box", dict(W=3)), ("gauss", dict(sigma_s=2.0))])
def test_one_slice_is_the_2d_filter(kind, kw):
    f = synthimg.gen1(70, 90, 11)[None]
    out, plan, f32 = _run(f, kind, 25.0, **kw)
    ref = G.gpa_alg2(f32[0], _w1(kind, kw), 25.0, plan.info.N, 127.5)
    assert np.abs(out[0] - ref).max() <= TOL


def _pairwise_at(f, vox, w1, sr, N):
    # eq. (GPA) at one voxel: its window is the zero-extended neighbourhood
    W = len(w1) // 2
    D, H, Wd = f.shape
    d, r, c = vox
    lo = [max(0, d - W), max(0, r - W), max(0, c - W)]
    hi = [min(D, d + W + 1), min(H, r + W + 1), min(Wd, c + W + 1)]
    sub = f[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
    return V.gpa_pairwise(sub, w1, sr, N, 127.5)[d - lo[0], r - lo[1], c - lo[2]]


def test_video_sampled():
    # 64 frames of 256^2 (4.2 Mvoxels), Gaussian sigma_s = 1.5 (W = 5), sampled voxels
    f = _vol(64, 256, 256, 20)
    out, plan, f32 = _run(f, "gauss", 30.0, sigma_s=1.5)
    rng = np.random.default_rng(21)
    vox = [(0, 0, 0), (63, 255, 255), (0, 255, 17), (31, 128, 0), (63, 3, 200)]
    vox += [tuple(int(v) for v in rng.integers([0, 0, 0], [64, 256, 256])) for _ in range(15)]
    w1 = _w1("gauss", dict(sigma_s=1.5))
    got = np.array([out[v] for v in vox])
    ref = np.array([_pairwise_at(f32, v, w1, 30.0, plan.info.N) for v in vox])
    print(f"N={plan.info.N} sampled max {np.abs(got - ref).max():.3e}", flush=True)
    assert np.abs(got - ref).max() <= TOL


def test_constant_volume_and_errors():
    torch, P = _mods()
    c = np.full((6, 40, 50), 133.0)
    out, _, _ = _run(c, "box", 10.0, W=4)
    assert np.abs(out - 133.0).max() <= TOL
    for kind, kw in (("gauss_rec", dict(sigma_s=2.0)), ("box", dict(W=3, grad=True)),
                     ("box", dict(W=33)), ("gauss", dict(sigma_s=2.0, joint=True))):
        with pytest.raises(P.BFError):
            P.VolumePlan(kind, 30.0, 4, 32, 32, **kw)
    import ctypes as C
    from paper_1603_08109_amd import _lib as L
    plan = P.VolumePlan("box", 30.0, 4, 32, 32, W=2)
    x = torch.zeros(4, 32, 32, device="cuda")
    y = torch.zeros_like(x)
    # a volume plan is not an image plan
    st = plan._lib.bf_forward(plan._h, C.c_void_p(x.data_ptr()), 32, C.c_void_p(y.data_ptr()), 32,
                              C.c_void_p(0), C.c_void_p(0))
    assert st == L.BF_EINVAL


MIRROR_CASES = [
    ("box", dict(W=2), 30.0, (5, 37, 45), 31),
    ("gauss", dict(sigma_s=1.5), 25.0, (6, 70, 66), 32),
    ("box", dict(W=5), 40.0, (3, 4, 90), 33),       # fewer slices and slice rows than the support
    ("gauss", dict(sigma_s=2.0), 15.0, (9, 20, 17), 34),
]


@pytest.mark.parametrize("kind,kw,sr,shape,seed", MIRROR_CASES)
def test_mirror_matches_oracle(kind, kw, sr, shape, seed):
    # reflection about every face: the row pass reflects columns, the in-slice column
    # FIR rows of the same slice, the depth FIR slices
    f = _vol(*shape, seed)
    out, plan, f32 = _run(f, kind, sr, mirror=True, **kw)
    ref = V.gpa_alg2_mirror(f32, _w1(kind, kw), sr, plan.info.N, 127.5)
    d = np.abs(out - ref)
    print(f"mirror {kind} {kw} sr={sr} {shape}: N={plan.info.N} max {d.max():.3e}", flush=True)
    assert d.max() <= TOL


@pytest.mark.parametrize("ss,sr,shape,mirror", [(1.0, 5.0, (4, 20, 30), False), (1.5, 6.0, (3, 16, 20), False),
                                                (1.0, 4.0, (2, 10, 12), True)])
def test_wide_range(ss, sr, shape, mirror):
    # T/sigma_r above 13: the float64-state row pass and depth fold, against eq. (GPA)
    # pair by pair in log space
    torch, P = _mods()
    f = _vol(*shape, 40)
    out, plan, f32 = _run(f, "gauss", sr, sigma_s=ss, mirror=mirror)
    w1 = _w1("gauss", dict(sigma_s=ss))
    ref = (V.gpa_pairwise_mirror if mirror else V.gpa_pairwise)(f32, w1, sr, plan.info.N, 127.5, wide=True)
    d = np.abs(out - ref)
    print(f"wide sigma_s={ss} sigma_r={sr} {shape} mirror={mirror}: N={plan.info.N} max {d.max():.3e}", flush=True)
    assert d.max() <= TOL


def test_plan_weight_and_order():
    torch, P = _mods()
    from oracle import order as O
    w1 = _w1("gauss", dict(sigma_s=2.0))
    plan = P.VolumePlan("gauss", 30.0, 4, 32, 32, sigma_s=2.0)
    assert plan.info.w0 == pytest.approx(V.w0(w1), rel=1e-12)
    assert plan.info.N == O.order_for_delta(1e-3, V.w0(w1), 127.5, 30.0)
