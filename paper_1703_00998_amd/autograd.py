"""torch.autograd.Function for the truncated approximation A_k = U_k U_k^T A
(Section 6.2, eq. Ak_randUTV) with the Gaussian G held fixed.

Forward and backward both run in the library (randutv_approx and
randutv_approx_backward): the backward recomputes every step's trailing
matrix from A and the saved reflectors and reverses the steps with its own
kernels.  torch only provides memory, the stream and the dtype conversion
(inputs of any float dtype are carried in FP64 storage; `prec` selects the
arithmetic of the large products as for randutv_factor).
"""
from __future__ import annotations

import torch

from . import binding as B


def _as_colmajor64(x):
    x = x.detach().to(torch.float64)
    return x.T.contiguous().T


class RandUTVApprox(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, G, b, q, k, prec="fp64"):
        Ad = _as_colmajor64(A)
        Gd = _as_colmajor64(G)
        Ak, Uk, tape = B.randutv_approx(Ad, Gd, b, q, k, prec=prec)
        ctx.save_for_backward(Ad, Gd, Uk, tape)
        ctx.cfg = (b, q, k, prec, A.dtype)
        return Ak.to(A.dtype)

    @staticmethod
    def backward(ctx, gAk):
        Ad, Gd, Uk, tape = ctx.saved_tensors
        b, q, k, prec, dtype = ctx.cfg
        Abar = B.randutv_approx_backward(Ad, Gd, b, q, k, Uk, tape, _as_colmajor64(gAk), prec=prec)
        return Abar.to(dtype), None, None, None, None, None


def randutv_approx(A, G, b, q, k, prec="fp64"):
    """A_k of A (m x n, cuda) with the packed Gaussian G (m x k); differentiable in A."""
    return RandUTVApprox.apply(A, G, b, q, k, prec)
