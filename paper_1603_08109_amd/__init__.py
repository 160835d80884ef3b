"""MI355X (gfx950) implementation of the Gaussian-Polynomial Approximation of
the bilateral filter (Chaudhury & Dabhade, arXiv 1603.08109).

The filter runs in hand-written HIP kernels behind the C ABI of
include/bf_gpa.h (libbfgpa.so, built in-tree by ``build.py``); this package is
a thin ctypes binding plus a torch.autograd wrapper.
"""
from ._lib import (BF_PATH_RECURSIVE, BF_PATH_STREAMED, BF_PATH_TILE,  # noqa: F401
                   BF_PATH_VOLUME, BF_PATH_WIDE, BFError)
from .api import (Batch, Plan, PlanInfo, VolumePlan, bf_order, forward_noalloc, image_range,  # noqa: F401
                  range_params, version)
from .autograd import BilateralGPA  # noqa: F401
