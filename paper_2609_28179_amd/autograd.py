"""torch.autograd.Function for the batched Cholesky solve X = A^{-1} B.

Forward: one fused factor-and-solve launch (glass_posv_batched) on copies of
A and B; the factor L and the solution X are saved.  Backward: one launch of
the hand-written adjoint kernel (glass_posv_adjoint_batched), which returns
dB = A^{-1} G and the symmetric dA = -(dB X^T + X dB^T) / 2.
"""
from __future__ import annotations

import torch

from . import glass


class CholeskySolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, force=None):
        L = A.detach().contiguous().clone()
        X = B.detach().contiguous().clone()
        _, X, info = glass.posv_(L, X, force=force)
        ctx.save_for_backward(L, X)
        ctx.force = force
        ctx.info = info
        return X

    @staticmethod
    def backward(ctx, G):
        L, X = ctx.saved_tensors
        dB, dA = glass.posv_adjoint(L, X, G.contiguous(), force=ctx.force)
        return dA, dB, None


def cholesky_solve(A, B, force=None):
    """X = A^{-1} B for a batch of SPD A [b,n,n] (lower triangle read) and B [b,n,r]."""
    return CholeskySolve.apply(A, B, force)
