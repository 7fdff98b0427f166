"""Weighted-quadrature row-wise assembly of IGA mass and stiffness matrices on MI355X.

Python binding of libwqa.so (C ABI in include/wqa.h).  Every step of the assembly and
of its adjoint runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch supplies device memory and the current HIP stream.

    import paper_1710_01048_amd as wqa
    sp = wqa.Space(dim=3, degree=3, n_elem=(96, 96, 96))     # default rules
    c = ...   # [N1, N2, N3] on sp.grid_axes("c")
    a = [...]  # a[k] on sp.grid_axes(k)
    M, K = sp.assemble_fused(c, a)                           # [rows, (2p+1)^3] each
    M, K = wqa.WQAssemble.apply(sp, c, *a)                   # differentiable

The method: Barton, Puzyrev, Deng, Calo, "Efficient mass and stiffness matrix
assembly via weighted Gaussian quadrature rules for B-splines" (arXiv 1710.01048):
each row i is integrated with its own weighted Gaussian rule whose weight is the
basis function B_i (Sec. 3), one direction at a time (eq:Decompo).
"""
from ._lib import (F32, F64, FINAL_DOT2, FINAL_F64, FINAL_PLAIN, MASS, STIFFNESS,
                   WQAError, lib, lib_path)
from .space import Space, WQAssemble

__all__ = ["Space", "WQAssemble", "WQAError", "lib", "lib_path", "MASS", "STIFFNESS", "F32", "F64",
           "FINAL_PLAIN", "FINAL_DOT2", "FINAL_F64"]
