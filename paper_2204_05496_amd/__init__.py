"""MI355X (gfx950) implementation of encrypted logistic-regression inference
under BFV: the fast matrix multiplication (Algorithm 1) of arXiv 2204.05496
and the standard encrypted matrix multiplication baseline.

The compute path lives in liblrhe.so (HIP kernels + C ABI, include/lrhe.h);
this package is the thin Python binding over it.
"""
from .bfv import Batch, Context, Keys, Model, Server, crt_combine, fixed_point, to_numpy_u32  # noqa: F401
from . import native  # noqa: F401

__all__ = ["Batch", "Context", "Keys", "Model", "Server", "crt_combine", "fixed_point", "to_numpy_u32", "native"]
