"""The plain streamed Gaussian forward with pre-split row-filtered images
(supports W >= 57, and every support on images of 4 Mpx or more, which run
64 orders per block): the row pass writes its outputs as three bfloat16
planes in groups of eight rows, round_up(W, 8) zero rows above the image,
and the column pass copies them into LDS with its taps shifted by
round_up(W, 8) - W rows.

Checked against the FP64 oracle (eq. GPA evaluated in Algorithm 2's
filtering form) and against the same plan's arithmetic on float32
row-filtered images: a plan with BF_FLAG_GRAD keeps those (its saved-state
forward needs them), and its plain forward runs the same products with the
split taken in the column pass instead of the row pass, so the two agree to
the float32 rounding of the split arithmetic (BETWEEN, as for the other
engine pairs).  Every shift 0..7 is covered, with heights that are not
multiples of the 16-row row tiles or the 256-row column tiles, widths that
are not multiples of the 16-column tiles, and images smaller than one tile.

Tolerance: max |GPU - oracle| <= 1e-3 on the 0-255 scale."""
import numpy as np
import pytest

import synthimg
from oracle import gpa as G
from oracle import kernels as K

pytestmark = pytest.mark.gpu
TOL = 1e-3
BETWEEN = 5e-4


def _run(f, W, sr, seed_ss=None):
    import torch
    import paper_1603_08109_amd as P
    assert torch.cuda.is_available()
    H, Wd = f.shape
    ss = W / 3.0 if seed_ss is None else seed_ss
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    a = P.Plan("gauss", sr, H, Wd, sigma_s=ss, W=W, engine="streamed")
    b = P.Plan("gauss", sr, H, Wd, sigma_s=ss, W=W, engine="streamed", grad=True)
    ya = a.forward(x)
    yb = b.forward(x)
    torch.cuda.synchronize()
    fx = x.cpu().numpy().astype(np.float64)
    return ya.cpu().numpy().astype(np.float64), yb.cpu().numpy().astype(np.float64), a, fx, ss


@pytest.mark.parametrize("W,shape", [(57, (97, 131)), (58, (300, 77)), (59, (261, 35)), (60, (17, 290)),
                                     (61, (130, 129)), (62, (256, 16)), (63, (40, 300)), (64, (270, 250))])
def test_presplit_every_shift(W, shape):
    f = synthimg.gen2(*shape, 500 + W)
    sr = 20.0 + (W % 3) * 10.0
    ya, yb, plan, fx, ss = _run(f, W, sr)
    ref = G.gpa_alg2(fx, K.taps1d("gauss", ss, W), sr, plan.info.N, 127.5)
    da, db = np.abs(ya - ref).max(), np.abs(yb - ref).max()
    dab = np.abs(ya - yb).max()
    print(f"W={W} shift={(-W) % 8} shape={shape} N={plan.info.N}: presplit {da:.3e} "
          f"float32 planes {db:.3e} between {dab:.3e}", flush=True)
    assert da <= TOL and db <= TOL
    assert dab <= BETWEEN


@pytest.mark.parametrize("shape", [(1, 1), (3, 200), (200, 2), (15, 15)])
def test_presplit_tiny_images(shape):
    # images smaller than one row tile, one column tile, or one pixel: the
    # window is mostly zero rows above and loads past the plane
    f = synthimg.gen1(*shape, 77)
    ya, yb, plan, fx, ss = _run(f, 75, 30.0, seed_ss=25.0)
    ref = G.gpa_alg2(fx, K.taps1d("gauss", ss, 75), 30.0, plan.info.N, 127.5)
    assert np.abs(ya - ref).max() <= TOL
    assert np.abs(ya - yb).max() <= BETWEEN


def test_presplit_two_calls_and_constant():
    # a constant image is a fixed point; a second call on other data reuses
    # the planes (rows past the image must still read as zeros)
    import torch
    import paper_1603_08109_amd as P
    H, Wd = 150, 190
    plan = P.Plan("gauss", 30.0, H, Wd, sigma_s=25.0, engine="streamed")
    c = torch.full((H, Wd), 173.0, dtype=torch.float32, device="cuda")
    yc = plan.forward(c)
    f = synthimg.gen2(H, Wd, 9)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    y = plan.forward(x)
    torch.cuda.synchronize()
    assert np.abs(yc.cpu().numpy() - 173.0).max() <= TOL
    fx = x.cpu().numpy().astype(np.float64)
    ref = G.gpa_alg2(fx, K.taps1d("gauss", 25.0), 30.0, plan.info.N, 127.5)
    assert np.abs(y.cpu().numpy().astype(np.float64) - ref).max() <= TOL


@pytest.mark.parametrize("W", [13, 30, 41])
def test_presplit_small_supports_4mpx(W):
    # images of 4 Mpx and more run 64 orders per block and pre-split planes at
    # every support: a band across the first 256-row column-tile seam and the
    # last rows, against the oracle on the band grown by W (exact there)
    import torch
    import paper_1603_08109_amd as P
    H = Wd = 2048
    f = synthimg.gen2(H, Wd, 700 + W)
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    ss = W / 3.0
    plan = P.Plan("gauss", 30.0, H, Wd, sigma_s=ss, W=W, engine="streamed")
    y = plan.forward(x)
    torch.cuda.synchronize()
    out = y.cpu().numpy().astype(np.float64)
    fx = x.cpu().numpy().astype(np.float64)
    w1 = K.taps1d("gauss", ss, W)
    for r0, r1, c0, c1 in [(254, 258, 0, Wd), (H - 3, H, Wd - 600, Wd)]:
        R0, R1, C0, C1 = max(0, r0 - W), min(H, r1 + W), max(0, c0 - W), min(Wd, c1 + W)
        ref = G.gpa_alg2(fx[R0:R1, C0:C1], w1, 30.0, plan.info.N, 127.5)[r0 - R0:r1 - R0, c0 - C0:c1 - C0]
        d = np.abs(out[r0:r1, c0:c1] - ref).max()
        print(f"W={W} band {r0}:{r1} x {c0}:{c1}: max {d:.3e}", flush=True)
        assert d <= TOL
