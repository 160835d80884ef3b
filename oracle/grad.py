"""Reference gradients of the GPA output, in float64.

The paper does not differentiate the filter; these are test references for
the adjoint the HIP library adds.  For a loss L with upstream gradient
gbar = dL/d(out), the quantities checked are the vector-Jacobian products

    dL/df (per pixel),   dL/d sigma_r,   dL/d sigma_s (Gaussian kernel only),

with N and the support W held fixed.

* ``vjp_autograd`` builds the N + 1 filtering form of the GPA (eqs. P, Q,
  PbyQ of Sec. 3) from plain torch CPU float64 operations (the separable
  zero-padded spatial filter is a pair of 1-D convolutions) and lets
  torch.autograd differentiate it.
* ``vjp_fd`` takes central finite differences of L = sum(gbar * out) with
  the numpy filtering form of ``oracle.gpa`` (a separate code path).
* ``mirror=True`` on either: the same with the reflecting
  border (image extended by reflection about its edges, edge samples
  repeated); autograd differentiates the reflection as the gather it is, the
  differences use the numpy ``oracle.mirror`` filter.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gpa as _gpa
from . import kernels as _k
from . import mirror as _mirror


def _taps_torch(kind: str, sigma_s, W: int):
    a = torch.arange(-W, W + 1, dtype=torch.float64)
    if kind == _k.BOX:
        return torch.ones_like(a)
    return torch.exp(-(a * a) / (2.0 * sigma_s * sigma_s))


def _filter_torch(F: torch.Tensor, w1: torch.Tensor) -> torch.Tensor:
    W = (w1.numel() - 1) // 2
    x = F[None, None]
    x = torch.nn.functional.conv2d(x, w1.view(1, 1, -1, 1), padding=(W, 0))
    x = torch.nn.functional.conv2d(x, w1.view(1, 1, 1, -1), padding=(0, W))
    return x[0, 0]


def gpa_torch(f: torch.Tensor, sigma_r: torch.Tensor, sigma_s, kind: str, W: int,
              N: int, T: float) -> torch.Tensor:
    """Eqs. (intImg), (spatialFiltering), (P), (Q), (PbyQ) (Sec. 3) in
    differentiable torch float64, with the centring of eq. (shift), t_c = T:
    F_n = exp(-u^2/2) u^n with u = (f - T)/sigma_r, each filtered once, and
    the sums of eqs. (P), (Q) with the weights u^n/n!."""
    w1 = _taps_torch(kind, sigma_s, W)
    u = (f - T) / sigma_r
    E = torch.exp(-0.5 * u * u)
    P = torch.zeros_like(f)
    Q = torch.zeros_like(f)
    c = torch.ones_like(f)          # u^n / n!, the product of the factors u/k
    Fbar_n = _filter_torch(E, w1)
    un = torch.ones_like(f)         # u^n
    for n in range(N):
        un = un * u
        Fbar_next = _filter_torch(E * un, w1)
        Q = Q + c * Fbar_n
        P = P + c * Fbar_next
        Fbar_n = Fbar_next
        c = c * (u / (n + 1))
    return sigma_r * (P / Q) + T


def vjp_autograd(f: np.ndarray, gbar: np.ndarray, kind: str, sigma_s, W: int,
                 sigma_r: float, N: int, T: float, mirror: bool = False):
    """(dL/df, dL/dsigma_r, dL/dsigma_s) by float64 autograd; dsigma_s is NaN for box.
    mirror: the image is first extended by W on each side by reflection (a gather
    with the reflected indices) and the output is the centre crop."""
    ft = torch.tensor(np.asarray(f, np.float64), requires_grad=True)
    sr = torch.tensor(float(sigma_r), dtype=torch.float64, requires_grad=True)
    ss = None
    if kind == _k.GAUSS:
        ss = torch.tensor(float(sigma_s), dtype=torch.float64, requires_grad=True)
    if mirror:
        H, Wd = ft.shape
        ri = torch.as_tensor(_mirror.reflect_index(np.arange(-W, H + W), H))
        ci = torch.as_tensor(_mirror.reflect_index(np.arange(-W, Wd + W), Wd))
        out = gpa_torch(ft[ri][:, ci], sr, ss, kind, W, N, T)[W:W + H, W:W + Wd]
    else:
        out = gpa_torch(ft, sr, ss, kind, W, N, T)
    L = (out * torch.tensor(np.asarray(gbar, np.float64))).sum()
    inputs = [ft, sr] + ([ss] if ss is not None else [])
    grads = torch.autograd.grad(L, inputs)
    dss = float(grads[2]) if ss is not None else float("nan")
    return grads[0].numpy(), float(grads[1]), dss


def _loss_np(f, gbar, kind, sigma_s, W, sigma_r, N, T, mirror=False):
    w1 = _k.taps1d(kind, sigma_s, W)
    alg2 = _mirror.gpa_alg2 if mirror else _gpa.gpa_alg2
    return float((np.asarray(gbar) * alg2(f, w1, sigma_r, N, T)).sum())


def vjp_fd(f: np.ndarray, gbar: np.ndarray, kind: str, sigma_s, W: int,
           sigma_r: float, N: int, T: float, pixels, h: float = 1e-3, mirror: bool = False):
    """Central differences (step h) of L = sum(gbar * out) with respect to
    f at the listed pixels, sigma_r, and sigma_s (Gaussian; W fixed); mirror:
    the reflecting-border filter of ``oracle.mirror``."""
    f = np.asarray(f, np.float64)
    args = (kind, sigma_s, W, sigma_r, N, T, mirror)
    df = []
    for (r, c) in pixels:
        fp = f.copy(); fp[r, c] += h
        fm = f.copy(); fm[r, c] -= h
        df.append((_loss_np(fp, gbar, *args) - _loss_np(fm, gbar, *args)) / (2 * h))
    dsr = (_loss_np(f, gbar, kind, sigma_s, W, sigma_r + h, N, T, mirror)
           - _loss_np(f, gbar, kind, sigma_s, W, sigma_r - h, N, T, mirror)) / (2 * h)
    dss = float("nan")
    if kind == _k.GAUSS:
        dss = (_loss_np(f, gbar, kind, sigma_s + h, W, sigma_r, N, T, mirror)
               - _loss_np(f, gbar, kind, sigma_s - h, W, sigma_r, N, T, mirror)) / (2 * h)
    return np.array(df), dsr, dss
