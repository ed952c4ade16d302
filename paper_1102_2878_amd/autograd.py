"""torch.autograd wrapper of the DFGT sums (argument marshalling only).

``gauss_sum_fn(q, r, h, eps)`` returns the (n_h, NQ) sums G~ as a
differentiable function of the query points ``q`` and the bandwidths ``h``.
When a gradient will be needed, the forward runs dfgt_gauss_sum_grad, which
returns the sums together with their exact derivatives (the same traversal,
the same interaction lists); the backward contracts those saved derivatives
with the incoming gradient through dfgt_gauss_sum_vjp.  So the backward
differentiates exactly the approximation the forward returned.  Without
gradients the forward is dfgt_gauss_sum.  The reference points are held
fixed: passing an ``r`` that requires grad raises (for the monochromatic case
pass ``r = q.detach()``).
"""
from __future__ import annotations

import numpy as np
import torch

from . import dfgt


class GaussSum(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, r, h, eps, leaf_size, precision):
        if r.requires_grad:
            raise NotImplementedError("gradients with respect to the reference points are not provided")
        qd = q.detach()
        Qt = dfgt.build_tree(qd, leaf_size=leaf_size)
        Rt = Qt if r.data_ptr() == qd.data_ptr() and r.shape == qd.shape else dfgt.build_tree(r, leaf_size=leaf_size)
        hv = np.asarray(h.detach().cpu(), dtype=np.float64).reshape(-1)
        need_q, _, need_h = ctx.needs_input_grad[:3]
        ctx.h_meta = (h.device, h.dtype, h.shape)
        if not (need_q or need_h):
            ctx.saved = (None, None)
            return dfgt.gauss_sum(Qt, Rt, hv, eps, precision=precision)
        G, Gh, Gq = dfgt.gauss_sum_grad(Qt, Rt, hv, eps, dh=need_h, dq=need_q, precision=precision)
        ctx.saved = (Gh, Gq)
        return G

    @staticmethod
    def backward(ctx, dG):
        Gh, Gq = ctx.saved
        need_q, _, need_h = ctx.needs_input_grad[:3]
        if not (need_q or need_h):
            return None, None, None, None, None, None
        dh, dq = dfgt.gauss_sum_vjp(dG.contiguous(), Gh if need_h else None, Gq if need_q else None)
        dev, dt, shp = ctx.h_meta
        gh = torch.as_tensor(dh, dtype=dt, device=dev).reshape(shp) if need_h else None
        return (dq if need_q else None), None, gh, None, None, None


def gauss_sum_fn(q, r, h, eps, leaf_size=0, precision=dfgt.PREC_MIXED):
    """Differentiable DFGT sums: (n_h, NQ) float64 CUDA tensor."""
    h = h if isinstance(h, torch.Tensor) else torch.as_tensor(h, dtype=torch.float64)
    return GaussSum.apply(q, r, h, float(eps), int(leaf_size), int(precision))
