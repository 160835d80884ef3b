"""GPU parity of the cross (joint) filter, bf_forward_joint, against the
float64 oracle (oracle.joint): the 2N-filtering form on small images, the
pair-by-pair form and the exact cross filter on a sampled 1024^2 image, the
plain filter when the guide is the input, and the error paths.
Tolerance: max |GPU - oracle| <= 1e-3 on the 0-255 scale."""
import numpy as np
import pytest

import synthimg
from oracle import joint as J
from oracle import kernels as K

pytestmark = pytest.mark.gpu
TOL = 1e-3


def _mods():
    import torch
    import paper_1603_08109_amd as P
    assert torch.cuda.is_available()
    return torch, P


def _run(f, h, kind, sr, **kw):
    torch, P = _mods()
    H, Wd = f.shape
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    g = torch.tensor(h, dtype=torch.float32, device="cuda")
    plan = P.Plan(kind, sr, H, Wd, joint=True, **kw)
    out = plan.forward_joint(x, g)
    torch.cuda.synchronize()
    return (out.cpu().numpy().astype(np.float64), plan, x.cpu().numpy().astype(np.float64),
            g.cpu().numpy().astype(np.float64))


CASES = [("box", dict(W=2), 30.0, (33, 47), 1), ("box", dict(W=9), 20.0, (120, 90), 2),
         ("gauss", dict(sigma_s=1.5), 25.0, (64, 70), 3), ("gauss", dict(sigma_s=3.0), 40.0, (100, 131), 4),
         ("gauss", dict(sigma_s=5.0), 15.0, (70, 66), 5)]


@pytest.mark.parametrize("kind,kw,sr,shape,seed", CASES)
def test_joint_matches_oracle(kind, kw, sr, shape, seed):
    f = synthimg.gen2(*shape, seed)
    h = synthimg.gen1(*shape, seed + 70)
    out, plan, f32, h32 = _run(f, h, kind, sr, **kw)
    w1 = K.taps1d(kind, kw.get("sigma_s"), kw.get("W") if kind == "box" else None)
    ref = J.gpa_joint_alg2(f32, h32, w1, sr, plan.info.N, 127.5)
    err = np.abs(out - ref).max()
    print(f"{kind} {kw} sr={sr} {shape} N={plan.info.N} tile={plan.info.tile_rows}: max {err:.3e}", flush=True)
    assert err <= TOL


def test_joint_workload_sampled():
    # 1024^2, Gaussian sigma_s = 5: the pair-by-pair form and the exact cross filter at sampled pixels
    f = synthimg.gen2(1024, 1024, 2100)
    h = synthimg.gen1(1024, 1024, 2101)
    out, plan, f32, h32 = _run(f, h, "gauss", 30.0, sigma_s=5.0)
    w2 = K.taps2d("gauss", 5.0)
    px = synthimg.sample_pixels(1024, 1024, 800, plan.info.W, 300, 2102)
    got = out[px[:, 0], px[:, 1]]
    o2 = J.gpa_joint_pairwise_at(f32, h32, px, w2, 30.0, plan.info.N, 127.5)
    o1 = J.direct_joint_bf_at(f32, h32, px, w2, 30.0)
    print(f"N={plan.info.N}: vs O2 {np.abs(got - o2).max():.3e}, vs O1 {np.abs(got - o1).max():.3e}", flush=True)
    assert np.abs(got - o2).max() <= TOL
    assert np.abs(got - o1).max() <= TOL


@pytest.mark.parametrize("shape", [(1, 1), (3, 200), (130, 2), (65, 65)])
def test_joint_ragged(shape):
    f = synthimg.gen2(*shape, 41)
    h = synthimg.gen1(*shape, 42)
    out, plan, f32, h32 = _run(f, h, "gauss", 20.0, sigma_s=2.0)
    ref = J.gpa_joint_alg2(f32, h32, K.taps1d("gauss", 2.0), 20.0, plan.info.N, 127.5)
    assert np.abs(out - ref).max() <= TOL


def test_guide_equal_input_matches_plain_filter():
    torch, P = _mods()
    f = synthimg.gen2(90, 110, 43)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    a = P.Plan("gauss", 30.0, 90, 110, sigma_s=3.0, joint=True).forward_joint(x, x)
    b = P.Plan("gauss", 30.0, 90, 110, sigma_s=3.0).forward(x)
    torch.cuda.synchronize()
    assert (a - b).abs().max().item() <= TOL


def test_joint_error_paths():
    torch, P = _mods()
    x = torch.zeros(20, 30, dtype=torch.float32, device="cuda")
    jp = P.Plan("box", 30.0, 20, 30, W=2, joint=True)
    with pytest.raises(P.BFError):
        jp.forward(x)
    with pytest.raises(P.BFError):
        P.Plan("box", 30.0, 20, 30, W=2).forward_joint(x, x.clone())
    with pytest.raises(P.BFError):
        P.Plan("box", 30.0, 20, 30, W=2, joint=True, grad=True)
    with pytest.raises(P.BFError):
        jp.forward_joint(x, x, out=x)  # out aliases the input
