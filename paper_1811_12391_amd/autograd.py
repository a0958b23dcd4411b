"""torch.autograd wrapper around the library's forward solve and its adjoint.

``roi_dose(solver, density, group_w, roi)`` returns the scalar response
R = sum_b sum_v roi[v] dose_b(v) as a float64 tensor whose gradient with
respect to ``density`` (one value per voxel, g/cm^3) and ``group_w`` (the
source spectrum, one weight per group) is the discrete adjoint computed by
``dct_adjoint`` (frozen fixup, reversed group order, transposed moment maps
and reverse-direction sweeps, ray back-projection of the uncollided flux).
The dose itself is Sec. II-A's collision-kerma tally; the gradient is an
addition built on the same discrete equations.

Only argument marshalling happens here: the forward solve, the response R
(``dct_roi_dose``) and the adjoint run in the HIP library; the densities and
weights enter through the library's host-buffer setters.  The adjoint needs
the kept state of the forward solve, so the solver must not be re-solved or
modified between forward and backward (the library reports DCT_ESTATE if it
was).
"""
from __future__ import annotations

import numpy as np
import torch

from . import dctsn


class _RoiDose(torch.autograd.Function):
    @staticmethod
    def forward(ctx, density, group_w, solver, roi, fwd_kw, adj_kw):
        solver.set_density(density.detach().cpu().numpy().astype(np.float64))
        solver.set_group_weights(group_w.detach().cpu().numpy().astype(np.float64))
        solver.solve(keep_adjoint=True, **fwd_kw)
        ctx.solver, ctx.roi, ctx.adj_kw = solver, np.asarray(roi, dtype=np.float64).reshape(-1), adj_kw
        ctx.dev = (density.device, group_w.device)
        R = dctsn.roi_dose(solver.h, solver.prob.phantom.C, ctx.roi)   # reduced in the library
        return torch.tensor(R, dtype=torch.float64, device=density.device)

    @staticmethod
    def backward(ctx, gR):
        a = ctx.solver.adjoint(ctx.roi, **ctx.adj_kw)
        s = float(gR)
        dd = torch.from_numpy(a.d_density * s).to(ctx.dev[0])
        dg = torch.from_numpy(a.d_group_w * s).to(ctx.dev[1])
        return dd, dg, None, None, None, None


def roi_dose(solver: "dctsn.Solver", density: torch.Tensor, group_w: torch.Tensor, roi, *, fwd=None,
             adj=None) -> torch.Tensor:
    """Differentiable ROI dose.  ``fwd`` / ``adj``: keyword options of the
    forward solve (precision, tol, fixed_iters, ...) and of the adjoint
    (tol, max_iter, fixed_iters)."""
    return _RoiDose.apply(density, group_w, solver, roi, dict(fwd or {}), dict(adj or {}))
