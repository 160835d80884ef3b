"""The adjoint (bf_backward) on the 4096^2 image of the large-support workload.

The output gradient gbar is zero except on a few 48 x 48 patches (centre of
the image, top edge, bottom-right corner).  The loss L = sum(gbar * out) then
depends only on the outputs inside the patches, and each of those depends on
the input within W of it.  So dL/df vanishes outside the patches grown by W,
and on each grown patch (a crop of the image, zero extension outside the
image as in the filter itself) the float64 autograd reference
oracle.grad.vjp_autograd gives dL/df exactly; the sigma gradients are the sums
of the crops' values.  The crops are far enough apart that no pixel lies in
two of them.

Covered: the fused adjoint tile (Gaussian sigma_s = 3, W = 9) and the
streamed adjoint (Gaussian sigma_s = 25 and box W = 75), at sigma_r = 10 and
30, with the forward state saved and recomputed.  Tolerance as for the small
adjoint tests: max |GPU - ref| <= 1e-3 max |ref| for dL/df, relative 1e-3 for
the sigma gradients; and dL/df exactly zero away from the grown patches.
"""
import functools

import numpy as np
import pytest

import synthimg
from oracle import grad as GR

pytestmark = pytest.mark.gpu
RTOL = 1e-3
H = Wd = 4096
PATCH = 48


@functools.lru_cache(maxsize=1)
def _image():
    return synthimg.gen2(H, Wd, 3000)


def _crop(r, c, W):
    return max(0, r - W), min(H, r + PATCH + W), max(0, c - W), min(Wd, c + PATCH + W)


def _check(kind, kw, sr, which, use_saved, seed):
    import torch
    import paper_1603_08109_amd as P
    assert torch.cuda.is_available()
    f = _image()
    patches = synthimg.grad_patches(H, Wd, PATCH, which)
    gbar = synthimg.patch_gbar(H, Wd, patches, PATCH, seed)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    g = torch.tensor(gbar, dtype=torch.float32, device="cuda")
    plan = P.Plan(kind, sr, H, Wd, grad=True, **kw)
    W, N = plan.info.W, plan.info.N
    print(f"# {kind} {kw} sigma_r={sr} W={W} N={N} patches={which} saved={use_saved}", flush=True)
    saved = plan.new_saved() if use_saved else None
    plan.forward(x, saved=saved)
    gin, gs = plan.backward(x, g, saved=saved)
    torch.cuda.synchronize()
    gin = gin.cpu().numpy().astype(np.float64)
    gs = gs.cpu().numpy()
    del saved, x, g
    f32 = np.asarray(f, np.float32).astype(np.float64)
    g32 = np.asarray(gbar, np.float32).astype(np.float64)
    outside = np.ones((H, Wd), dtype=bool)
    dsr = dss = 0.0
    worst = scale = 0.0
    sq = 0.0
    cnt = 0
    for (r, c) in patches:
        r0, r1, c0, c1 = _crop(r, c, W)
        outside[r0:r1, c0:c1] = False
        df, a, b = GR.vjp_autograd(f32[r0:r1, c0:c1], g32[r0:r1, c0:c1], kind, kw.get("sigma_s"), W, sr, N, 127.5)
        d = gin[r0:r1, c0:c1] - df
        worst = max(worst, float(np.abs(d).max()))
        scale = max(scale, float(np.abs(df).max()))
        sq += float((d * d).sum())
        cnt += d.size
        dsr += a
        dss += b
    assert scale > 0.0
    rms = (sq / cnt) ** 0.5
    print(f"df max {worst / scale:.2e} rms {rms / scale:.2e} (of max |ref| {scale:.3e}); "
          f"dsr {gs[0]:.8e} vs {dsr:.8e}; dss {gs[1]:.8e} vs {dss:.8e}", flush=True)
    assert np.count_nonzero(gin[outside]) == 0
    assert worst <= RTOL * scale
    assert abs(gs[0] - dsr) <= RTOL * abs(dsr)
    if kind == "gauss":
        assert abs(gs[1] - dss) <= RTOL * abs(dss)
    else:
        assert np.isnan(gs[1])


ALL = ("centre", "edge", "corner")


@pytest.mark.parametrize("sr,use_saved", [(10.0, True), (30.0, False)])
def test_fused_adjoint_4096(sr, use_saved):
    _check("gauss", dict(sigma_s=3.0), sr, ALL, use_saved, 7100 + int(sr))


@pytest.mark.parametrize("kind,kw,sr,which", [
    ("gauss", dict(sigma_s=25.0), 30.0, ALL),
    ("gauss", dict(sigma_s=25.0), 10.0, ("corner",)),
    ("box", dict(W=75), 30.0, ALL),
    ("box", dict(W=75), 10.0, ("edge",)),
])
def test_streamed_adjoint_4096(kind, kw, sr, which):
    _check(kind, kw, sr, which, sr < 20.0, 7200 + int(sr))


def test_streamed_adjoint_4096_recompute():
    # the streamed adjoint recomputing its forward state at the full size
    _check("gauss", dict(sigma_s=10.0), 30.0, ("corner", "centre"), False, 7300)
