"""torch.autograd wrapper of the DFGT sums (argument marshalling only).

``gauss_sum_fn(q, r, h, eps)`` returns the (n_h, NQ) sums of dfgt_gauss_sum as a
differentiable function of the query points ``q`` and the bandwidths ``h``;
its backward calls dfgt_gauss_sum_backward, which recomputes the same
approximation together with its exact derivatives in the HIP library.  The
reference points are held fixed: passing an ``r`` that requires grad raises
(for the monochromatic case pass ``r = q.detach()``).
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
        G = dfgt.gauss_sum(Qt, Rt, hv, eps, precision=precision)
        ctx.trees = (Qt, Rt)
        ctx.hv, ctx.eps, ctx.precision = hv, eps, precision
        ctx.h_meta = (h.device, h.dtype, h.shape)
        return G

    @staticmethod
    def backward(ctx, dG):
        Qt, Rt = ctx.trees
        need_q, _, need_h = ctx.needs_input_grad[:3]
        if not (need_q or need_h):
            return None, None, None, None, None, None
        dh, dq = dfgt.gauss_sum_backward(Qt, Rt, ctx.hv, ctx.eps, dG.contiguous(), want_dh=need_h, want_dq=need_q,
                                         precision=ctx.precision)
        dev, dt, shp = ctx.h_meta
        gh = torch.as_tensor(dh, dtype=dt, device=dev).reshape(shp) if need_h else None
        return (dq if need_q else None), None, gh, None, None, None


def gauss_sum_fn(q, r, h, eps, leaf_size=0, precision=dfgt.PREC_MIXED):
    """Differentiable DFGT sums: (n_h, NQ) float64 CUDA tensor."""
    h = h if isinstance(h, torch.Tensor) else torch.as_tensor(h, dtype=torch.float64)
    return GaussSum.apply(q, r, h, float(eps), int(leaf_size), int(precision))
