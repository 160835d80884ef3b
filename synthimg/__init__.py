"""Seeded synthetic inputs shared by the HIP path's tests and the CPU oracle.

The paper evaluates on a set of eight 512x512 8-bit grayscale photographs
(Sec. 4, Fig. "dataset"); that set is not available here, so every workload
is synthetic.  This module only draws pixels and per-image parameters: it
holds none of the bilateral-filter arithmetic, and neither the oracle nor
the product package is imported from here.

Generators
----------
gen1(H, W, seed)
    Piecewise-constant 16x16 blocks with levels ~ U[0, 255], plus i.i.d.
    Gaussian noise of standard deviation 20, clipped to [0, 255] (float64).
    Draw order with ``numpy.random.default_rng(seed)``: block levels first,
    then the noise field.
gen2(H, W, seed)
    gen1 plus a smooth ramp 40*sin(2*pi*(i/H + j/W)) added to the blocks
    before the noise, then clipped.
batch_params(count, seed)
    Per-image sizes and filter parameters of the uneven batch workload:
    width ~ U{64..1024}, height ~ U{64..768}, sigma_s ~ U[2, 15],
    sigma_r ~ U[10, 60].
clean_blocks(H, W, seed)
    The noise-free block image that gen1(H, W, seed) starts from (the
    regression target of the differentiable workload).
clean2(H, W, seed)
    The noise-free image (blocks plus ramp, clipped) that gen2(H, W, seed)
    starts from.
grad_patches, patch_gbar
    Patches of an image and an output gradient supported on them (checks of
    the adjoint on crops of large images).

Seeds: workload k, image b uses ``seed = 1000*k + b``.
"""
from __future__ import annotations

import numpy as np

BLOCK = 16
NOISE_SD = 20.0
RAMP_AMPLITUDE = 40.0


def _levels(rng: np.random.Generator, H: int, W: int) -> np.ndarray:
    gh = -(-H // BLOCK)
    gw = -(-W // BLOCK)
    lv = rng.uniform(0.0, 255.0, size=(gh, gw))
    return np.kron(lv, np.ones((BLOCK, BLOCK)))[:H, :W]


def clean_blocks(H: int, W: int, seed: int) -> np.ndarray:
    """Noise-free piecewise-constant image underlying gen1(H, W, seed)."""
    rng = np.random.default_rng(seed)
    return _levels(rng, H, W)


def gen1(H: int, W: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    base = _levels(rng, H, W)
    noise = rng.normal(0.0, NOISE_SD, size=(H, W))
    return np.clip(base + noise, 0.0, 255.0)


def ramp(H: int, W: int) -> np.ndarray:
    i = np.arange(H, dtype=np.float64)[:, None]
    j = np.arange(W, dtype=np.float64)[None, :]
    return RAMP_AMPLITUDE * np.sin(2.0 * np.pi * (i / H + j / W))


def clean2(H: int, W: int, seed: int) -> np.ndarray:
    """Noise-free image underlying gen2(H, W, seed): blocks plus ramp, clipped."""
    rng = np.random.default_rng(seed)
    return np.clip(_levels(rng, H, W) + ramp(H, W), 0.0, 255.0)


def gen2(H: int, W: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    base = _levels(rng, H, W) + ramp(H, W)
    noise = rng.normal(0.0, NOISE_SD, size=(H, W))
    return np.clip(base + noise, 0.0, 255.0)


def batch_params(count: int, seed: int):
    """List of dicts {height, width, sigma_s, sigma_r, seed} for an uneven batch."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        w = int(rng.integers(64, 1025))
        h = int(rng.integers(64, 769))
        ss = float(rng.uniform(2.0, 15.0))
        sr = float(rng.uniform(10.0, 60.0))
        out.append(dict(height=h, width=w, sigma_s=ss, sigma_r=sr, seed=seed + 1 + b))
    return out


def sample_pixels(H: int, W: int, count: int, border: int, border_count: int,
                  seed: int) -> np.ndarray:
    """Seeded pixel sample used to check full-size results pixel by pixel.

    `count` uniform pixels, `border_count` uniform pixels from the band of
    width `border` along the image edge, and the four corners; deduplicated,
    returned as an (M, 2) int64 array of (row, col) in raster order."""
    rng = np.random.default_rng(seed)
    mask = np.zeros((H, W), dtype=bool)
    mask[rng.integers(0, H, size=count), rng.integers(0, W, size=count)] = True
    b = max(0, min(border, H, W))
    if b > 0 and border_count > 0:
        band = np.zeros((H, W), dtype=bool)
        band[:b, :] = True
        band[-b:, :] = True
        band[:, :b] = True
        band[:, -b:] = True
        br, bc = np.nonzero(band)
        pick = rng.integers(0, br.size, size=border_count)
        mask[br[pick], bc[pick]] = True
    mask[0, 0] = mask[0, -1] = mask[-1, 0] = mask[-1, -1] = True
    rr, cc = np.nonzero(mask)
    return np.stack([rr, cc], axis=1).astype(np.int64)


def grad_patches(H: int, W: int, size: int, which=("centre", "edge", "corner")) -> list:
    """Top-left (row, col) of square `size` x `size` patches of an H x W image:
    'centre' (middle of the image), 'edge' (on the top edge, a quarter of the
    way across) and 'corner' (the bottom-right corner)."""
    pos = {"centre": ((H - size) // 2, (W - size) // 2),
           "edge": (0, max(0, W // 4 - size // 2)),
           "corner": (H - size, W - size)}
    return [pos[k] for k in which]


def patch_gbar(H: int, W: int, patches, size: int, seed: int) -> np.ndarray:
    """Output gradient that is zero except on the listed size x size patches,
    where it takes seeded values in [-0.5, 0.5] (gen2 levels / 255 - 0.5).
    With such a gradient, dL/d(input) and the parameter gradients of a filter
    with support W depend only on the patches grown by W, so a reference can
    be computed on crops of that size."""
    g = np.zeros((H, W))
    for k, (r, c) in enumerate(patches):
        g[r:r + size, c:c + size] = gen2(size, size, seed + k) / 255.0 - 0.5
    return g
