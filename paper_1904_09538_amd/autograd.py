"""torch.autograd.Function over the DG differentiation operator.

Forward and backward both run in libdgdiff's HIP kernels (dgdiff_apply and
dgdiff_backward); this module only routes tensors and honours
needs_input_grad.  FP32 and FP64 tensors on the current GPU.
"""
from __future__ import annotations

import torch

from . import _lib


class DGDiffFn(torch.autograd.Function):
    """out[m][e][i] = sum_j D[m][i][j] u[e][j]."""

    @staticmethod
    def forward(ctx, D, u):
        D = D.contiguous()
        u = u.contiguous()
        ctx.save_for_backward(D, u)
        return _lib.dgdiff_apply(D, u)

    @staticmethod
    def backward(ctx, g):
        D, u = ctx.saved_tensors
        want_D, want_u = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (want_D or want_u):
            return None, None
        gu, gD = _lib.dgdiff_backward(D, u, g.contiguous(), want_u=want_u, want_D=want_D)
        return gD, gu


def dgdiff(D, u):
    return DGDiffFn.apply(D, u)
