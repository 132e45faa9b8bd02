"""z(f^T) after T PDR-ESO passes as a differentiable function of (u, d).

`residual_after_sweeps(graph, u, d, T, checkpoint)` runs T passes of
Algorithm 1 with the exact edge subproblem (Algorithm 2) in FP64 from f = 0
and returns the objective of Expression 8 at the last iterate. Its backward is
the reverse-mode gradient pdr_adjoint computes on the GPU in the same call
(Section 4.4's pass map differentiated through the branch each arc takes; at a
tie between branches it is one of the one-sided derivatives).

This module only marshals: the forward pass and the gradient both come from
the library's kernels. Importing it imports torch first, so the library binds
to torch's HIP runtime.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ESO, FP64, Context, PdrError


class ResidualAfterSweeps(torch.autograd.Function):
    """autograd.Function over pdr_adjoint. Inputs u (m) and d (K) are float64
    tensors on any device; the graph (n, CSR row_ptr and heads col, sources s,
    sinks t) and T, checkpoint are constants. Returns a 0-dim float64 tensor on
    u's device."""

    @staticmethod
    def forward(ctx, u, d, graph, T, checkpoint):
        if u.dtype != torch.float64 or d.dtype != torch.float64:
            raise TypeError("u and d must be float64 tensors")
        n, row_ptr, col, s, t = graph
        uh = u.detach().to("cpu").numpy()
        dh = d.detach().to("cpu").numpy()
        want_grad = any(ctx.needs_input_grad[:2])
        with Context(n, row_ptr, col, uh, s, t, dh, method=ESO, precision=FP64) as c:
            if want_grad:
                z, gu, gd = c.adjoint(int(T), int(checkpoint))
            else:  # no gradient wanted: the T passes and the objective only
                c.sweep(int(T))
                res = c.residual()
                if res["status"] != "PDR_OK":
                    raise PdrError(5 if res["status"] == "PDR_ERR_NUMERIC" else 3, "pdr_residual")
                z = res["z"]
        if want_grad:
            ctx.save_for_backward(torch.from_numpy(np.ascontiguousarray(gu)).to(u.device),
                                  torch.from_numpy(np.ascontiguousarray(gd)).to(d.device))
        return torch.tensor(z, dtype=torch.float64, device=u.device)

    @staticmethod
    def backward(ctx, gz):
        gu, gd = ctx.saved_tensors
        gu_out = gz.to(gu.device) * gu if ctx.needs_input_grad[0] else None
        gd_out = gz.to(gd.device) * gd if ctx.needs_input_grad[1] else None
        return gu_out, gd_out, None, None, None


def residual_after_sweeps(graph, u, d, T: int, checkpoint: int = 16):
    """z(f^T) for capacities u and demands d on `graph`, differentiable in u
    and d. `graph` is (n, row_ptr, col, s, t) or any object with those
    attributes (an instance record)."""
    if not isinstance(graph, tuple):
        graph = (graph.n, graph.row_ptr, graph.col, graph.s, graph.t)
    return ResidualAfterSweeps.apply(u, d, graph, int(T), int(checkpoint))
