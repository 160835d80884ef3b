"""Forward parity on the 4096^2 image of the large-support workload, on row
bands that cross the seams of each engine's work decomposition.

Each engine that the planner picks at 4096^2 is checked on its own shape:
  * the fused tile on the vector ALUs (Gaussian sigma_s = 3 and box W = 10):
    tiles of 64 columns x tile_rows rows;
  * the box column strips (256 columns at W = 30, 512 columns at W = 75),
    cut into row segments (the plan reports both);
  * the split-bfloat16 row pass writing its outputs split, with the column
    pass on them (Gaussian sigma_s = 10 and 25; 4096^2 plans run 64 orders
    per block): 16 x 256 row tiles, column tiles of 16 columns x 256 rows.
A band of rows [r0, r1) and columns [c0, c1) is compared with Algorithm 2
(oracle.gpa.gpa_alg2) evaluated on the crop grown by W on every side (clipped
to the image).  Every output of the band has its whole window inside that crop
or outside the image, so the crop gives the band's values exactly.  The bands
straddle a row seam (tile rows, strip segments) and run across many column
seams; the last rows and columns of the image are checked too.
Tolerance: max |GPU - oracle| <= 1e-3 on the 0..255 scale.
"""
import functools

import numpy as np
import pytest

import synthimg
from oracle import gpa as G
from oracle import kernels as K

pytestmark = pytest.mark.gpu
TOL = 1e-3
H = Wd = 4096


@functools.lru_cache(maxsize=1)
def _image():
    return synthimg.gen2(H, Wd, 3000)


def _bands(kind, W, info):
    if info.path == 0:  # fused tile: seam between the first two tile rows, full width
        seam_r, seam_c = info.tile_rows, 64
    elif kind == "box":  # column strips: row segments and output columns per strip, as the plan reports them
        seam_r, seam_c = info.tile_rows, info.tile_cols
    else:  # streamed Gaussian: 16-row row-pass tiles, 256-row column-pass tiles
        seam_r, seam_c = 256, 256
    # narrow supports: full-width bands; wide ones: 3+ column seams (cost)
    width = Wd if W <= 30 else 3 * seam_c + 40
    return [(seam_r - 2, seam_r + 2, 0, width),
            (3 * seam_r - 1, 3 * seam_r + 1, Wd - width, Wd),
            (H - 2, H, Wd - min(width, 700), Wd)]


CASES = [
    ("gauss", dict(sigma_s=3.0), 10.0, "tile"),
    ("box", dict(W=10), 10.0, "tile"),
    ("box", dict(W=30), 30.0, "streamed"),
    ("box", dict(W=75), 30.0, "streamed"),
    ("gauss", dict(sigma_s=10.0), 30.0, "streamed"),
    ("gauss", dict(sigma_s=25.0), 50.0, "streamed"),
]


@pytest.mark.parametrize("kind,kw,sr,engine", CASES)
def test_band_parity_4096(kind, kw, sr, engine):
    import torch
    import paper_1603_08109_amd as P
    assert torch.cuda.is_available()
    f = _image()
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    plan = P.Plan(kind, sr, H, Wd, **kw)
    W, N = plan.info.W, plan.info.N
    print(f"# {kind} {kw} sigma_r={sr} W={W} N={N} path={plan.info.path} tile_rows={plan.info.tile_rows} "
          f"tile_cols={plan.info.tile_cols}", flush=True)
    assert (plan.info.path == 0) == (engine == "tile")
    if kind == "box" and engine == "streamed":  # the strip decomposition is reported
        assert plan.info.tile_rows > 0 and plan.info.tile_cols == (512 if W >= 48 else 256) - 2 * W
    out = plan.forward(x)
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.float64)
    del x
    f32 = np.asarray(f, np.float32).astype(np.float64)
    w1 = K.taps1d(kind, kw.get("sigma_s"), kw.get("W"))
    for (r0, r1, c0, c1) in _bands(kind, W, plan.info):
        R0, R1, C0, C1 = max(0, r0 - W), min(H, r1 + W), max(0, c0 - W), min(Wd, c1 + W)
        ref = G.gpa_alg2(f32[R0:R1, C0:C1], w1, sr, N, 127.5)[r0 - R0:r1 - R0, c0 - C0:c1 - C0]
        d = out[r0:r1, c0:c1] - ref
        print(f"band rows {r0}:{r1} cols {c0}:{c1}: max {np.abs(d).max():.2e} rms {np.sqrt(np.mean(d * d)):.2e}",
              flush=True)
        assert np.abs(d).max() <= TOL
