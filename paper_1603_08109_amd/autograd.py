"""torch.autograd wrapper around bf_forward / bf_backward.

``BilateralGPA`` holds sigma_r (and sigma_s for the Gaussian kernel) as
parameters; the order N and support W are fixed at construction (they are
integers and are held constant when differentiating).  The forward saves
three per-pixel values (Q, P/Q and the coefficient-derivative term) for the
adjoint; the N+1 auxiliary images are recomputed inside the adjoint kernel,
never stored.  With ``mirror=True`` (reflecting border) nothing is saved: the
adjoint recomputes its state on the image extended by reflection.
"""
from __future__ import annotations

import torch

from .api import Plan


class _GPAFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, image, sigma_r, sigma_s, module):
        plan = module._plan_for(image)
        saved = None if module.mirror else plan.new_saved()
        out = plan.forward(image.detach(), saved=saved)
        ctx.plan = plan
        ctx.save_for_backward(image, saved)
        ctx.has_ss = sigma_s is not None and sigma_s.requires_grad
        return out

    @staticmethod
    def backward(ctx, gout):
        image, saved = ctx.saved_tensors
        plan = ctx.plan
        gin, gs = plan.backward(image.detach(), gout.contiguous(), saved=saved, want_sigma=True)
        gsr = gs[0].to(torch.float32).reshape(())
        gss = gs[1].to(torch.float32).reshape(()) if ctx.has_ss else None
        return gin, gsr, gss, None


class BilateralGPA(torch.nn.Module):
    """Differentiable GPA bilateral filter on (H, W) float32 CUDA images."""

    def __init__(self, kernel: str, sigma_r: float, sigma_s: float | None = None, W: int = 0,
                 N: int | None = None, delta: float = 1e-3, T: float = 127.5,
                 center: float | None = None, mirror: bool = False):
        super().__init__()
        self.kernel = kernel
        self.mirror = mirror
        self.sigma_r = torch.nn.Parameter(torch.tensor(float(sigma_r)))
        self.sigma_s = torch.nn.Parameter(torch.tensor(float(sigma_s))) if kernel != "box" else None
        self.W = W
        self.delta, self.T, self.center = delta, T, center
        self._N = N
        self._plans = {}

    def _plan_for(self, image: torch.Tensor) -> Plan:
        H, Wd = image.shape
        key = (H, Wd, float(self.sigma_r.detach()),
               float(self.sigma_s.detach()) if self.sigma_s is not None else None)
        plan = self._plans.get(key)
        if plan is None:
            kw = dict(W=self.W, T=self.T, center=self.center, delta=self.delta, grad=True, mirror=self.mirror)
            if self._N is not None:
                kw["N"] = self._N
            if self.sigma_s is not None:
                kw["sigma_s"] = float(self.sigma_s.detach())
            plan = Plan(self.kernel, float(self.sigma_r.detach()), H, Wd, **kw)
            if self._N is None:
                self._N = plan.info.N       # hold N fixed from here on
                self.W = plan.info.W        # and the support
            self._plans = {key: plan}
        return plan

    def forward(self, image: torch.Tensor) -> torch.Tensor:
        return _GPAFunction.apply(image, self.sigma_r, self.sigma_s, self)
