"""GPU parity of the recursive-Gaussian path (BF_GAUSS_REC) against the FP64
oracle twin (``oracle.recursive``: the filter as its plain definition, the
matrix product K_H F K_W^T with K[i, j] = h(|i - j|)).

Tolerance: max |GPU - oracle| <= 1e-3 on the 0-255 scale, oracle in float64
on the float32-rounded input at the same N.  Shapes span one chunk, several
chunks with ragged tails along both axes, lines of one sample, a full 4096
row and column (the longest scans the bench shape has), and the 4096^2 bench
shape at sampled pixels."""
import numpy as np
import pytest

import synthimg
from oracle import recursive as R

pytestmark = pytest.mark.gpu
TOL = 1e-3


def _mods():
    import torch
    import paper_1603_08109_amd as P
    assert torch.cuda.is_available()
    return torch, P


def _forward(f, sr, ss, **kw):
    torch, P = _mods()
    H, Wd = f.shape
    x = torch.tensor(f, dtype=torch.float32, device="cuda")
    plan = P.Plan("gauss_rec", sr, H, Wd, sigma_s=ss, **kw)
    assert plan.info.path == P.BF_PATH_RECURSIVE
    out = plan.forward(x)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), plan, x.cpu().numpy().astype(np.float64)


def _report(name, d):
    print(f"{name}: max {np.abs(d).max():.3e} rms {np.sqrt(np.mean(d * d)):.3e}", flush=True)


CASES = [
    (1.0, 30.0, (37, 45), 1),
    (3.0, 30.0, (96, 130), 2),
    (3.0, 10.0, (64, 64), 3),
    (10.0, 30.0, (150, 170), 4),
    (25.0, 20.0, (140, 133), 5),
    (60.0, 30.0, (90, 300), 6),
    (0.5, 25.0, (17, 33), 7),
    (5.0, 50.0, (257, 16), 8),
]


@pytest.mark.parametrize("ss,sr,shape,seed", CASES)
def test_matches_oracle(ss, sr, shape, seed):
    f = synthimg.gen2(*shape, seed)
    out, plan, f32 = _forward(f, sr, ss)
    ref = R.gpa_alg2(f32, ss, sr, plan.info.N, 127.5)
    print(f"sigma_s={ss} sr={sr} {shape}: N={plan.info.N}", flush=True)
    _report("gpu-oracle", out - ref)
    assert np.abs(out - ref).max() <= TOL


@pytest.mark.parametrize("shape", [(1, 1), (1, 200), (200, 1), (3, 3), (16, 16), (5, 64), (65, 129)])
def test_ragged_and_tiny(shape):
    f = synthimg.gen1(*shape, 31)
    out, plan, f32 = _forward(f, 25.0, 2.0)
    ref = R.gpa_alg2(f32, 2.0, 25.0, plan.info.N, 127.5)
    assert np.abs(out - ref).max() <= TOL, shape


@pytest.mark.parametrize("shape", [(8, 4096), (4096, 8)])
def test_long_lines(shape):
    # 256 chunks per line: eight scan steps
    f = synthimg.gen2(*shape, 41)
    out, plan, f32 = _forward(f, 30.0, 25.0)
    ref = R.gpa_alg2(f32, 25.0, 30.0, plan.info.N, 127.5)
    _report(f"{shape}", out - ref)
    assert np.abs(out - ref).max() <= TOL


def test_direct_filter_and_constants():
    # converges to the direct filter with this kernel; constants are fixed points
    torch, P = _mods()
    f = synthimg.gen1(24, 28, 51)
    out, plan, f32 = _forward(f, 30.0, 2.0, delta=1e-4)
    exact = R.direct_bf(f32, 2.0, 30.0)
    _report("gpu-direct", out - exact)
    assert np.abs(out - exact).max() <= 2e-3
    c = np.full((40, 50), 91.0)
    out, _, _ = _forward(c, 10.0, 7.0)
    assert np.abs(out - 91.0).max() <= TOL


@pytest.mark.parametrize("ss,sr", [(3.0, 50.0), (25.0, 30.0)])
def test_full_size_sampled(ss, sr):
    # the 4096^2 shape, sampled pixels (corners, borders, interior)
    f = synthimg.gen2(4096, 4096, 4100)
    out, plan, f32 = _forward(f, sr, ss)
    px = np.array([[0, 0], [0, 4095], [4095, 0], [4095, 4095], [2048, 2047], [17, 3001], [3999, 5],
                   [1024, 1024], [77, 4000], [2500, 1]])
    ref = R.gpa_alg2_at(f32, px, ss, sr, plan.info.N, 127.5)
    got = out[px[:, 0], px[:, 1]]
    print(f"N={plan.info.N}", flush=True)
    _report("gpu-oracle", got - ref)
    assert np.abs(got - ref).max() <= TOL


def test_unsupported_combinations():
    torch, P = _mods()
    for kw in (dict(grad=True), dict(mirror=True), dict(joint=True), dict(engine="valu")):
        with pytest.raises(P.BFError):
            P.Plan("gauss_rec", 30.0, 64, 64, sigma_s=2.0, **kw)
    plan = P.Plan("gauss_rec", 30.0, 32, 32, sigma_s=2.0)
    x = torch.zeros(32, 32, device="cuda")
    with pytest.raises(P.BFError):
        plan.forward(x, saved=torch.empty(3 * 32 * 32, device="cuda"))
