"""torch.autograd.Function around the forward and the hand-written adjoint.

C = TotalConv.apply(alm, blm, cosbeta, lmax, mbmax) computes
C_{mb,msky}(beta_j) = sum_l conj(b_{l,mb}) d^l_{mb,msky}(beta_j) s_{l,msky}
(eq. convdef of Prezeau & Reinecke, Sec. 4.1).  C is complex-linear in the sky
and conjugate-linear in the beam; backward returns PyTorch's gradients
(dL/dRe + i dL/dIm) for both, computed by the adjoint kernel, which recomputes
d^l on the fly.  For a real a_{l,0} the caller keeps the real part of its
gradient.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding


class TotalConv(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alm, blm, cosbeta, lmax, mbmax):
        x = np.ascontiguousarray(cosbeta, dtype=np.float64)
        C = _binding.totalconv_fwd(lmax, mbmax, x, alm.detach().contiguous(), blm.detach().contiguous())
        ctx.save_for_backward(alm, blm)
        ctx.x = x
        ctx.lmax = lmax
        ctx.mbmax = mbmax
        return C

    @staticmethod
    def backward(ctx, gC):
        alm, blm = ctx.saved_tensors
        want_a, want_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (want_a or want_b):
            return None, None, None, None, None
        ga, gb = _binding.totalconv_adj(ctx.lmax, ctx.mbmax, ctx.x, alm.detach().contiguous(),
                                        blm.detach().contiguous(), gC.contiguous(),
                                        want_alm=want_a, want_blm=want_b)
        return ga, gb, None, None, None


def totalconv(alm, blm, cosbeta, lmax: int, mbmax: int):
    return TotalConv.apply(alm, blm, cosbeta, lmax, mbmax)
