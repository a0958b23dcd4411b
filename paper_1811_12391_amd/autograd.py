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
(``dct_roi_dose``) and the adjoint run in the HIP library.  A density tensor
on the GPU stays there: the library copies it on the device
(``dct_set_density_dev``) and writes the density gradient into a GPU tensor
(``dct_adjoint_dev``).  A host density goes through the host-buffer setters.
The group weights (G numbers that define the source with its position and
collimation) always pass through ``dct_set_source``.  The adjoint needs the
kept state of the forward solve, so the solver must not be re-solved or
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
        if density.is_cuda:
            solver.set_density(density.detach().to(torch.float64).contiguous().reshape(-1))
        else:
            solver.set_density(density.detach().numpy().astype(np.float64).reshape(-1))
        solver.set_group_weights(group_w.detach().cpu().numpy().astype(np.float64))
        solver.solve(keep_adjoint=True, **fwd_kw)
        ctx.solver, ctx.roi, ctx.adj_kw = solver, np.asarray(roi, dtype=np.float64).reshape(-1), adj_kw
        ctx.dev = (density.device, group_w.device)
        ctx.shape = density.shape
        R = dctsn.roi_dose(solver.h, solver.prob.phantom.C, ctx.roi)   # reduced in the library
        return torch.tensor(R, dtype=torch.float64, device=density.device)

    @staticmethod
    def backward(ctx, gR):
        s = float(gR)
        if ctx.dev[0].type == "cuda":
            dev = ctx.dev[0]
            p = ctx.solver.prob
            roi_t = torch.from_numpy(ctx.roi).to(dev)
            dd = torch.empty(p.phantom.C, dtype=torch.float64, device=dev)
            dg = torch.empty(p.G, dtype=torch.float64, device=dev)
            ctx.solver.adjoint_dev(roi_t, dd, dg, **ctx.adj_kw)
            return (dd * s).reshape(ctx.shape), (dg * s).to(ctx.dev[1]), None, None, None, None
        a = ctx.solver.adjoint(ctx.roi, **ctx.adj_kw)
        dd = torch.from_numpy(a.d_density * s).reshape(ctx.shape).to(ctx.dev[0])
        dg = torch.from_numpy(a.d_group_w * s).to(ctx.dev[1])
        return dd, dg, None, None, None, None


def roi_dose(solver: "dctsn.Solver", density: torch.Tensor, group_w: torch.Tensor, roi, *, fwd=None,
             adj=None) -> torch.Tensor:
    """Differentiable ROI dose.  ``fwd`` / ``adj``: keyword options of the
    forward solve (precision, tol, fixed_iters, ...) and of the adjoint
    (tol, max_iter, fixed_iters)."""
    return _RoiDose.apply(density, group_w, solver, roi, dict(fwd or {}), dict(adj or {}))
