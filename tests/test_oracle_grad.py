"""Pins for oracle.grad: float64 autograd through Algorithm 2 against central
finite differences of the separate numpy Algorithm 2."""
import numpy as np
import pytest

import synthimg
from oracle import grad as GR
from oracle import kernels as K


@pytest.mark.parametrize("kind,sigma_s,W", [(K.BOX, None, 2), (K.GAUSS, 1.5, 5)])
def test_autograd_matches_fd(kind, sigma_s, W):
    f = synthimg.gen1(14, 13, 3)
    target = synthimg.clean_blocks(14, 13, 3)
    N, sr, T = 30, 30.0, 127.5
    # gbar of an MSE loss against the clean target, evaluated at the oracle output
    from oracle import gpa
    out = gpa.gpa_alg2(f, K.taps1d(kind, sigma_s, W), sr, N, T)
    gbar = 2.0 * (out - target) / out.size
    df, dsr, dss = GR.vjp_autograd(f, gbar, kind, sigma_s, W, sr, N, T)
    px = np.array([[0, 0], [3, 4], [7, 12], [13, 6]])
    fd_f, fd_sr, fd_ss = GR.vjp_fd(f, gbar, kind, sigma_s, W, sr, N, T, px, h=1e-3)
    scale = np.abs(df).max()
    assert np.allclose(df[px[:, 0], px[:, 1]], fd_f, rtol=1e-5, atol=1e-7 * scale)
    assert dsr == pytest.approx(fd_sr, rel=1e-5, abs=1e-9)
    if kind == K.GAUSS:
        assert dss == pytest.approx(fd_ss, rel=1e-5, abs=1e-9)
    else:
        assert np.isnan(dss)


@pytest.mark.parametrize("kind,sigma_s,W,shape", [(K.BOX, None, 2, (14, 13)), (K.GAUSS, 1.5, 5, (4, 13))])
def test_mirror_autograd_matches_fd(kind, sigma_s, W, shape):
    # the reflecting border: autograd through the reflected gather against central differences
    # of the numpy mirror filter, at corners, edges and inside; (4, 13) with W = 5 reflects the
    # rows more than once, so one pixel's value reaches a window through several reflections
    f = synthimg.gen1(*shape, 5)
    gbar = synthimg.gen2(*shape, 6) / 255.0 - 0.5
    N, sr, T = 30, 30.0, 127.5
    df, dsr, dss = GR.vjp_autograd(f, gbar, kind, sigma_s, W, sr, N, T, mirror=True)
    H, Wd = shape
    px = np.array([[0, 0], [H - 1, Wd - 1], [0, Wd // 2], [H // 2, 0], [H // 2, Wd - 2], [H - 1, 3]])
    fd_f, fd_sr, fd_ss = GR.vjp_fd(f, gbar, kind, sigma_s, W, sr, N, T, px, h=1e-3, mirror=True)
    scale = np.abs(df).max()
    assert np.allclose(df[px[:, 0], px[:, 1]], fd_f, rtol=1e-5, atol=1e-7 * scale)
    assert dsr == pytest.approx(fd_sr, rel=1e-5, abs=1e-9)
    if kind == K.GAUSS:
        assert dss == pytest.approx(fd_ss, rel=1e-5, abs=1e-9)
    # the border changes the gradient: it is not the zero-border one
    dz = GR.vjp_autograd(f, gbar, kind, sigma_s, W, sr, N, T)[0]
    assert np.abs(dz - df).max() > 1e-3 * scale
