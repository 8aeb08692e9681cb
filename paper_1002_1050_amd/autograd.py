"""torch.autograd.Function around the forward and the hand-written adjoint.

C = TotalConv.apply(alm, blm, beta, lmax, mbmax) computes
C_{mb,msky}(beta_j) = sum_l conj(b_{l,mb}) d^l_{mb,msky}(beta_j) s_{l,msky}
(eq. convdef of Prezeau & Reinecke, Sec. 4.1) on the colatitudes beta (host);
TotalConvX takes the ring cosines instead.  C is complex-linear in the sky
and conjugate-linear in the beam; backward returns PyTorch's gradients
(dL/dRe + i dL/dIm) for both, computed by the adjoint kernel, which recomputes
d^l on the fly.  For a real a_{l,0} the caller keeps the real part of its
gradient.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding


class TotalConvX(torch.autograd.Function):
    """C from the sky and beam on ring cosines cosbeta (the library's rings, see
    _binding.rings_from_beta); backward by the adjoint kernel."""

    @staticmethod
    def forward(ctx, alm, blm, cosbeta, lmax, mbmax):
        x = np.ascontiguousarray(cosbeta, dtype=np.float64)
        C = _binding.totalconv_fwd_x(lmax, mbmax, x, alm.detach().contiguous(), blm.detach().contiguous())
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
        ga, gb = _binding.totalconv_adj_x(ctx.lmax, ctx.mbmax, ctx.x, alm.detach().contiguous(),
                                        blm.detach().contiguous(), gC.contiguous(),
                                        want_alm=want_a, want_blm=want_b)
        return ga, gb, None, None, None


class TotalConv(TotalConvX):
    """C from the sky and beam on colatitudes beta: the rings are formed once
    (tc_rings_from_beta) and the forward and the adjoint run on them."""

    @staticmethod
    def forward(ctx, alm, blm, beta, lmax, mbmax):
        return TotalConvX.forward(ctx, alm, blm, _binding.rings_from_beta(beta), lmax, mbmax)


def totalconv(alm, blm, beta, lmax: int, mbmax: int):
    return TotalConv.apply(alm, blm, beta, lmax, mbmax)


class TotalConvPolX(torch.autograd.Function):
    """Polarised form on ring cosines: TotalConvPolX.apply(mode, cosbeta, lmax, mbmax, alm_0, ..,
    alm_{n-1}, blm_0, .., blm_{n-1}) for n = 1..3 (temperature, gradient, curl) pairs; returns
    one C per pair (TC_POL_SEPARATE) or the one summed C (TC_POL_SUM), as a tuple."""

    @staticmethod
    def forward(ctx, mode, cosbeta, lmax, mbmax, *tensors):
        n = len(tensors) // 2
        if len(tensors) != 2 * n or not 1 <= n <= 3:
            raise ValueError("pass 1 to 3 sky tensors followed by as many beam tensors")
        x = np.ascontiguousarray(cosbeta, dtype=np.float64)
        alms = [t.detach().contiguous() for t in tensors[:n]]
        blms = [t.detach().contiguous() for t in tensors[n:]]
        outs = _binding.totalconv_fwd_pol_x(lmax, mbmax, x, alms, blms, mode)
        ctx.save_for_backward(*tensors)
        ctx.x, ctx.lmax, ctx.mbmax, ctx.mode, ctx.n = x, lmax, mbmax, mode, n
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grads):
        tensors = ctx.saved_tensors
        n = ctx.n
        want_a = any(ctx.needs_input_grad[4:4 + n])
        want_b = any(ctx.needs_input_grad[4 + n:4 + 2 * n])
        none = (None,) * 4
        if not (want_a or want_b):
            return none + (None,) * (2 * n)
        shape = (2 * ctx.mbmax + 1, ctx.lmax + 1, ctx.x.size)
        cot = [g if g is not None else torch.zeros(shape, dtype=torch.complex128, device=tensors[0].device)
               for g in grads]
        ga, gb = _binding.totalconv_adj_pol_x(ctx.lmax, ctx.mbmax, ctx.x, [t.detach().contiguous() for t in tensors[:n]],
                                            [t.detach().contiguous() for t in tensors[n:]],
                                            [g.contiguous() for g in cot], ctx.mode,
                                            want_alm=want_a, want_blm=want_b)
        return none + tuple(ga) + tuple(gb)


class TotalConvPol(TotalConvPolX):
    """Polarised form on colatitudes: TotalConvPol.apply(mode, beta, lmax, mbmax, alm_0, ..,
    blm_{n-1}); the rings are formed once (tc_rings_from_beta)."""

    @staticmethod
    def forward(ctx, mode, beta, lmax, mbmax, *tensors):
        return TotalConvPolX.forward(ctx, mode, _binding.rings_from_beta(beta), lmax, mbmax, *tensors)
