"""Python binding of the C ABI: argument marshalling only.

Every step of the filter runs in the HIP library; torch supplies device
memory and the current stream.  Names follow the C entry points:
``bf_order``, ``Plan`` (bf_plan / bf_forward / bf_backward / bf_destroy) and
``Batch`` (bf_batch_plan / bf_batch_forward / bf_batch_tune / ...).
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import torch

from . import _lib as L

_RULES = {"lambertw": L.BF_NRULE_LAMBERTW, "alg1": L.BF_NRULE_ALG1, "poisson": L.BF_NRULE_POISSON}
_KERNELS = {"box": L.BF_BOX, "gauss": L.BF_GAUSS, "gaussian": L.BF_GAUSS, "gauss_rec": L.BF_GAUSS_REC}
_ENGINES = {None: 0, "auto": 0, "valu": L.BF_FLAG_TILE_VALU,
            "streamed": L.BF_FLAG_STREAMED}
PATHS = {L.BF_PATH_TILE: "valu", L.BF_PATH_STREAMED: "streamed",
         L.BF_PATH_RECURSIVE: "recursive", L.BF_PATH_VOLUME: "volume", L.BF_PATH_WIDE: "wide"}


@dataclass
class PlanInfo:
    N: int
    W: int
    w0: float
    eps: float
    lam: float
    kernel_bound: float
    guaranteed_delta: float
    tile_rows: int
    tile_cols: int
    workspace_bytes: int
    path: int = 0
    status: int = 0


def make_params(kernel: str, sigma_r: float, *, sigma_s: float | None = None, W: int = 0,
                T: float = 127.5, center: float | None = None, N: int = 0, delta: float = 1e-3,
                n_rule: str = "lambertw", height: int = 0, width: int = 0,
                fp32_accum: bool = False, grad: bool = False, streamed: bool = False,
                joint: bool = False, mirror: bool = False, engine: str | None = None,
                mfma_fp32: bool = False) -> L.bf_params:
    """bf_params; `engine` forces the forward engine: "valu" (fused tile on the
    vector ALUs) or "streamed"; `mfma_fp32`
    keeps the streamed Gaussian passes on plain float32 matrix-core products."""
    p = L.bf_params()
    p.kernel = _KERNELS[kernel]
    p.sigma_s = float(sigma_s) if sigma_s is not None else 0.0
    p.W = int(W)
    p.sigma_r = float(sigma_r)
    p.T = float(T)
    p.center = float("nan") if center is None else float(center)
    p.N = int(N)
    p.delta = float(delta)
    p.n_rule = _RULES[n_rule]
    p.height = int(height)
    p.width = int(width)
    p.flags = ((L.BF_FLAG_FP32_ACCUM if fp32_accum else 0) | (L.BF_FLAG_GRAD if grad else 0)
               | (L.BF_FLAG_STREAMED if streamed else 0) | (L.BF_FLAG_JOINT if joint else 0)
               | (L.BF_FLAG_MIRROR if mirror else 0) | _ENGINES[engine]
               | (L.BF_FLAG_MFMA_FP32 if mfma_fp32 else 0))
    return p


def _info(i: L.bf_plan_info, status: int = 0) -> PlanInfo:
    return PlanInfo(i.N, i.W, i.w0, i.eps, i.lambda_, i.kernel_bound, i.guaranteed_delta,
                    i.tile_rows, i.tile_cols, i.workspace_bytes, i.path, status)


def bf_order(kernel: str, sigma_r: float, **kw) -> PlanInfo:
    """Host-only planning (N, W, w0, eps, bounds); no device access."""
    lib = L.load()
    p = make_params(kernel, sigma_r, **kw)
    info = L.bf_plan_info()
    st = L.check(lib.bf_order(C.byref(p), C.byref(info)), "bf_order")
    return _info(info, st)


def _stream_handle(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


def _check_image(t: torch.Tensor, H: int, W: int, name: str):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 CUDA (HIP) tensor")
    if t.dim() != 2 or t.shape[0] != H or t.shape[1] != W:
        raise ValueError(f"{name} must have shape ({H}, {W}), got {tuple(t.shape)}")
    if t.stride(1) != 1:
        raise ValueError(f"{name} rows must be contiguous")


class VolumePlan:
    """A volume (or video) of `depth` slices of height x width (bf_plan_volume /
    bf_forward_volume); the kernel is w1 x w1 x w1."""

    def __init__(self, kernel: str, sigma_r: float, depth: int, height: int, width: int, **kw):
        self._lib = L.load()
        self.kernel = kernel
        self.depth, self.height, self.width = int(depth), int(height), int(width)
        self.params = make_params(kernel, sigma_r, height=height, width=width, **kw)
        h = C.c_void_p()
        st = L.check(self._lib.bf_plan_volume(C.byref(self.params), self.depth, C.byref(h)), "bf_plan_volume")
        self._h = h
        info = L.bf_plan_info()
        L.check(self._lib.bf_plan_get_info(self._h, C.byref(info)), "bf_plan_get_info")
        self.info = _info(info, st)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.bf_destroy(h)
            self._h = None

    def forward(self, inp: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """`inp`: (depth, height, width) float32 CUDA tensor with contiguous rows and
        slices stacked (stride(0) == height * stride(1))."""
        D, H, W = self.depth, self.height, self.width
        for t, name in ((inp, "input"), (out, "output")):
            if t is None:
                continue
            if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32:
                raise TypeError(f"{name} must be a float32 CUDA (HIP) tensor")
            stacked = D == 1 or t.stride(0) == H * t.stride(1)  # a size-1 dim's stride is arbitrary
            if tuple(t.shape) != (D, H, W) or t.stride(2) != 1 or not stacked:
                raise ValueError(f"{name} must be ({D}, {H}, {W}) with stacked slices, got {tuple(t.shape)}")
        if out is None:
            out = torch.empty_like(inp)
        L.check(self._lib.bf_forward_volume(self._h, C.c_void_p(inp.data_ptr()), inp.stride(1),
                                            C.c_void_p(out.data_ptr()), out.stride(1), _stream_handle(stream)),
                "bf_forward_volume")
        return out


class Plan:
    """One image size and parameter set (bf_plan)."""

    def __init__(self, kernel: str, sigma_r: float, height: int, width: int, **kw):
        self._lib = L.load()
        self.kernel = kernel
        self.height, self.width = int(height), int(width)
        self.params = make_params(kernel, sigma_r, height=height, width=width, **kw)
        h = C.c_void_p()
        st = L.check(self._lib.bf_plan(C.byref(self.params), C.byref(h)), "bf_plan")
        self._h = h
        info = L.bf_plan_info()
        L.check(self._lib.bf_plan_get_info(self._h, C.byref(info)), "bf_plan_get_info")
        self.info = _info(info, st)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.bf_destroy(h)
            self._h = None

    def clone(self) -> "Plan":
        """Same parameters, separate device workspace (bf_plan_clone_workspace)."""
        c = Plan.__new__(Plan)
        c._lib = self._lib
        c.kernel = self.kernel
        c.height, c.width = self.height, self.width
        c.params = self.params
        h = C.c_void_p()
        st = L.check(self._lib.bf_plan_clone_workspace(self._h, C.byref(h)), "bf_plan_clone_workspace")
        c._h = h
        info = L.bf_plan_info()
        L.check(self._lib.bf_plan_get_info(c._h, C.byref(info)), "bf_plan_get_info")
        c.info = _info(info, st)
        return c

    def new_saved(self) -> torch.Tensor:
        return torch.empty(3 * self.height * self.width, dtype=torch.float32, device="cuda")

    def forward(self, inp: torch.Tensor, out: torch.Tensor | None = None,
                saved: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        _check_image(inp, self.height, self.width, "input")
        if out is None:
            out = torch.empty_like(inp)
        _check_image(out, self.height, self.width, "output")
        sp = C.c_void_p(saved.data_ptr()) if saved is not None else C.c_void_p(0)
        L.check(self._lib.bf_forward(self._h, C.c_void_p(inp.data_ptr()), inp.stride(0),
                                     C.c_void_p(out.data_ptr()), out.stride(0), sp,
                                     _stream_handle(stream)), "bf_forward")
        return out

    def forward_joint(self, inp: torch.Tensor, guide: torch.Tensor, out: torch.Tensor | None = None,
                      stream=None) -> torch.Tensor:
        """Cross (joint) filter of `inp` with the range kernel on `guide` (plan built with joint=True)."""
        _check_image(inp, self.height, self.width, "input")
        _check_image(guide, self.height, self.width, "guide")
        if out is None:
            out = torch.empty_like(inp)
        _check_image(out, self.height, self.width, "output")
        L.check(self._lib.bf_forward_joint(self._h, C.c_void_p(inp.data_ptr()), inp.stride(0),
                                           C.c_void_p(guide.data_ptr()), guide.stride(0),
                                           C.c_void_p(out.data_ptr()), out.stride(0), _stream_handle(stream)),
                "bf_forward_joint")
        return out

    def backward(self, inp: torch.Tensor, grad_out: torch.Tensor, saved: torch.Tensor | None = None,
                 grad_in: torch.Tensor | None = None, want_sigma: bool = True, stream=None):
        """Returns (dL/din, tensor([dL/dsigma_r, dL/dsigma_s]) float64 or None)."""
        _check_image(inp, self.height, self.width, "input")
        _check_image(grad_out, self.height, self.width, "grad_out")
        if grad_in is None:
            grad_in = torch.empty_like(inp)
        gs = torch.empty(2, dtype=torch.float64, device=inp.device) if want_sigma else None
        L.check(self._lib.bf_backward(
            self._h, C.c_void_p(inp.data_ptr()), inp.stride(0), C.c_void_p(grad_out.data_ptr()),
            grad_out.stride(0), C.c_void_p(saved.data_ptr() if saved is not None else 0),
            C.c_void_p(grad_in.data_ptr()), grad_in.stride(0),
            C.c_void_p(gs.data_ptr() if gs is not None else 0), _stream_handle(stream)), "bf_backward")
        return grad_in, gs


class Batch:
    """Many images of uneven size in one persistent launch (bf_batch_*)."""

    def __init__(self, per_image: list[dict]):
        self._lib = L.load()
        self.count = len(per_image)
        arr = (L.bf_params * self.count)()
        self.shapes = []
        for i, d in enumerate(per_image):
            d = dict(d)
            kernel = d.pop("kernel")
            sigma_r = d.pop("sigma_r")
            arr[i] = make_params(kernel, sigma_r, **d)
            self.shapes.append((int(d["height"]), int(d["width"])))
        h = C.c_void_p()
        self.status = L.check(self._lib.bf_batch_plan(self.count, arr, C.byref(h)), "bf_batch_plan")
        self._h = h
        st = (C.c_int32 * self.count)()
        ns = (C.c_int32 * self.count)()
        L.check(self._lib.bf_batch_status(self._h, st, ns), "bf_batch_status")
        self.image_status = list(st)
        self.N = list(ns)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.bf_batch_destroy(h)
            self._h = None

    def _arrays(self, inputs, outputs):
        n = self.count
        if len(inputs) != n or len(outputs) != n:
            raise ValueError("one input and one output per image")
        ip = (C.c_void_p * n)()
        op = (C.c_void_p * n)()
        ipt = (C.c_int64 * n)()
        opt = (C.c_int64 * n)()
        for i, (a, b) in enumerate(zip(inputs, outputs)):
            H, W = self.shapes[i]
            _check_image(a, H, W, f"input[{i}]")
            _check_image(b, H, W, f"output[{i}]")
            ip[i], op[i] = a.data_ptr(), b.data_ptr()
            ipt[i], opt[i] = a.stride(0), b.stride(0)
        return ip, ipt, op, opt

    def new_saved(self) -> list:
        """Per-image forward-state buffers (3 * height * width float32) for forward/backward(saved=...)."""
        return [torch.empty(3 * H * W, dtype=torch.float32, device="cuda") for H, W in self.shapes]

    def _saved_array(self, saved):
        n = self.count
        if len(saved) != n:
            raise ValueError("one saved buffer per image")
        arr = (C.c_void_p * n)()
        for i, t in enumerate(saved):
            H, W = self.shapes[i]
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() < 3 * H * W:
                raise ValueError(f"saved[{i}] must be a contiguous CUDA float32 tensor of 3*{H}*{W} elements")
            arr[i] = t.data_ptr()
        return arr

    def forward(self, inputs, outputs=None, saved=None, stream=None):
        """saved: None, or new_saved() buffers that receive each image's forward state."""
        if outputs is None:
            outputs = [torch.empty_like(x) for x in inputs]
        ip, ipt, op, opt = self._arrays(inputs, outputs)
        if saved is None:
            L.check(self._lib.bf_batch_forward(self._h, ip, ipt, op, opt, _stream_handle(stream)),
                    "bf_batch_forward")
        else:
            L.check(self._lib.bf_batch_forward_saved(self._h, ip, ipt, op, opt, self._saved_array(saved),
                                                     _stream_handle(stream)), "bf_batch_forward_saved")
        return outputs

    def backward(self, inputs, grad_outs, grad_ins=None, want_sigma: bool = True, saved=None, stream=None):
        """Returns (list of dL/din_i, float64 tensor (count, 2) of [dL/dsigma_r, dL/dsigma_s] or None).
        saved: None (the forward state is recomputed) or the buffers forward(saved=...) filled."""
        n = self.count
        if len(inputs) != n or len(grad_outs) != n:
            raise ValueError("one input and one output gradient per image")
        if grad_ins is None:
            grad_ins = [torch.empty_like(x) for x in inputs]
        ip = (C.c_void_p * n)()
        ipt = (C.c_int64 * n)()
        gp = (C.c_void_p * n)()
        gpt = (C.c_int64 * n)()
        op = (C.c_void_p * n)()
        opt = (C.c_int64 * n)()
        for i, (a, g, o) in enumerate(zip(inputs, grad_outs, grad_ins)):
            H, W = self.shapes[i]
            _check_image(a, H, W, f"input[{i}]")
            _check_image(g, H, W, f"grad_out[{i}]")
            _check_image(o, H, W, f"grad_in[{i}]")
            ip[i], ipt[i] = a.data_ptr(), a.stride(0)
            gp[i], gpt[i] = g.data_ptr(), g.stride(0)
            op[i], opt[i] = o.data_ptr(), o.stride(0)
        dev = inputs[0].device
        gs = torch.empty(n, 2, dtype=torch.float64, device=dev) if want_sigma else None
        gsp = C.c_void_p(gs.data_ptr() if gs is not None else 0)
        if saved is None:
            L.check(self._lib.bf_batch_backward(self._h, ip, ipt, gp, gpt, op, opt, gsp, _stream_handle(stream)),
                    "bf_batch_backward")
        else:
            L.check(self._lib.bf_batch_backward_saved(self._h, ip, ipt, gp, gpt, self._saved_array(saved), op, opt,
                                                      gsp, _stream_handle(stream)), "bf_batch_backward_saved")
        return grad_ins, gs

    def get_info(self) -> dict:
        """bf_batch_get_info: how the batch runs (persistent / streamed images, LDS,
        workspace, graph launches of the forward)."""
        i = L.bf_batch_info()
        L.check(self._lib.bf_batch_get_info(self._h, C.byref(i)), "bf_batch_get_info")
        return {k: getattr(i, k) for k, _ in L.bf_batch_info._fields_}

    def tune(self, inputs, outputs, stream=None) -> int:
        ip, ipt, op, opt = self._arrays(inputs, outputs)
        ch = C.c_int32(-1)
        L.check(self._lib.bf_batch_tune(self._h, ip, ipt, op, opt, _stream_handle(stream), C.byref(ch)),
                "bf_batch_tune")
        return ch.value


def forward_noalloc(kernel: str, sigma_r: float, inp: torch.Tensor, out: torch.Tensor | None = None,
                    stream=None, **kw) -> torch.Tensor:
    """bf_forward_noalloc: the plain forward without a plan; the library keeps
    the constant tables in its static device array (no device allocation in the
    call; pass `out` to avoid torch allocating one)."""
    H, Wd = inp.shape
    _check_image(inp, H, Wd, "inp")
    if out is None:
        out = torch.empty_like(inp)
    _check_image(out, H, Wd, "out")
    p = make_params(kernel, sigma_r, height=H, width=Wd, **kw)
    lib = L.load()
    L.check(lib.bf_forward_noalloc(C.byref(p), C.c_void_p(inp.data_ptr()), inp.stride(0),
                                   C.c_void_p(out.data_ptr()), out.stride(0), _stream_handle(stream)),
            "bf_forward_noalloc")
    return out


def image_range(img: torch.Tensor, stream=None) -> torch.Tensor:
    """Device float32 tensor [min, max] of a 2-D float32 image (bf_image_range)."""
    if not isinstance(img, torch.Tensor) or img.device.type != "cuda" or img.dtype != torch.float32:
        raise TypeError("image must be a float32 CUDA (HIP) tensor")
    if img.dim() != 2 or img.stride(1) != 1:
        raise ValueError("image must be 2-D with contiguous rows")
    mm = torch.empty(2, dtype=torch.float32, device=img.device)
    lib = L.load()
    L.check(lib.bf_image_range(C.c_void_p(img.data_ptr()), img.stride(0), img.shape[0], img.shape[1],
                               C.c_void_p(mm.data_ptr()), _stream_handle(stream)), "bf_image_range")
    return mm


def range_params(vmin: float, vmax: float) -> dict:
    """center and T for a plan from a data range (keeps |f - center| <= T)."""
    T = max(0.5 * (float(vmax) - float(vmin)), 1e-6)
    return {"center": 0.5 * (float(vmax) + float(vmin)), "T": T}


def version() -> str:
    return L.load().bf_version().decode()
