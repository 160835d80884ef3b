"""Data-driven range (bf_image_range) and planning with the centre and
half-range taken from the data: the reduction is exact (min and max are
selections), and plans built from the data range keep the accuracy target
against the float64 oracle while needing fewer orders."""
import numpy as np
import pytest

import synthimg
from oracle import bf as B
from oracle import gpa as G
from oracle import kernels as K

pytestmark = pytest.mark.gpu


def _mods():
    import torch
    import paper_1603_08109_amd as P
    assert torch.cuda.is_available()
    return torch, P


@pytest.mark.parametrize("shape", [(1, 1), (3, 1000), (517, 333), (2048, 2048)])
def test_image_range_exact(shape):
    torch, P = _mods()
    rng = np.random.default_rng(shape[0] * 7 + shape[1])
    a = (rng.standard_normal(shape) * 300.0 - 20.0).astype(np.float32)
    a[rng.integers(0, shape[0]), rng.integers(0, shape[1])] = np.nan
    if a.size > 1:
        assert np.isnan(a).sum() == 1
    big = torch.zeros(shape[0], shape[1] + 13, dtype=torch.float32, device="cuda")
    big[:, :shape[1]] = torch.from_numpy(a).cuda()
    mm = P.image_range(big[:, :shape[1]]).cpu().numpy()
    if a.size == 1:
        assert mm[0] == np.inf and mm[1] == -np.inf
    else:
        assert mm[0] == np.nanmin(a) and mm[1] == np.nanmax(a)


def _narrow(shape, seed, lo, hi):
    f = synthimg.gen2(*shape, seed)
    return lo + (hi - lo) * f / 255.0


@pytest.mark.parametrize("kind,kw,sr", [("gauss", dict(sigma_s=2.0), 20.0), ("box", dict(W=3), 15.0)])
def test_data_range_plan_meets_delta(kind, kw, sr):
    torch, P = _mods()
    f = _narrow((48, 56), 11, 70.0, 170.0)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    mm = P.image_range(x).cpu().numpy()
    rp = P.range_params(mm[0], mm[1])
    plan = P.Plan(kind, sr, 48, 56, **rp, **kw)
    default = P.Plan(kind, sr, 48, 56, **kw)
    assert plan.info.N < default.info.N
    out = plan.forward(x)
    torch.cuda.synchronize()
    f32 = x.cpu().numpy().astype(np.float64)
    w2 = K.taps2d(kind, kw.get("sigma_s"), kw.get("W") if kind == "box" else None)
    o2 = G.gpa_pairwise(f32, w2, sr, plan.info.N, rp["center"])
    o1 = B.direct_bf(f32, w2, sr)
    got = out.cpu().numpy().astype(np.float64)
    print(f"N {plan.info.N} (default {default.info.N}); vs O2 {np.abs(got - o2).max():.2e}, "
          f"vs O1 {np.abs(got - o1).max():.2e}", flush=True)
    assert np.abs(got - o2).max() <= 1e-3
    assert np.abs(got - o1).max() <= 1e-3  # the delta = 1e-3 guarantee with the data range


def test_small_sigma_r_with_data_range():
    # sigma_r = 5 is outside the float32 domain for T = 127.5 (lambda = 650:
    # only the wide-range float64-state path, N = 796) but a float32 path with a
    # far lower order for a data range of width 80 (lambda = 64)
    torch, P = _mods()
    full = P.Plan("gauss", 5.0, 40, 40, sigma_s=1.5)
    assert full.info.path == P.BF_PATH_WIDE
    with pytest.raises(P.BFError):
        P.Plan("box", 5.0, 40, 40, W=2)
    f = _narrow((40, 40), 12, 100.0, 180.0)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    mm = P.image_range(x).cpu().numpy()
    rp = P.range_params(mm[0], mm[1])
    plan = P.Plan("gauss", 5.0, 40, 40, sigma_s=1.5, **rp)
    assert plan.info.path != P.BF_PATH_WIDE and plan.info.N < full.info.N // 4
    out = plan.forward(x)
    torch.cuda.synchronize()
    f32 = x.cpu().numpy().astype(np.float64)
    o1 = B.direct_bf(f32, K.taps2d("gauss", 1.5), 5.0)
    assert np.abs(out.cpu().numpy() - o1).max() <= 1e-3
