"""torch.autograd binding of the GICP cost (Eq. 4 with the Cauchy rho of
Eq. 5) and its hand-written gradient kernel.

Argument marshalling only: the forward is far_gicp_linearize (cost), the
backward is far_gicp_gradient, which searches the correspondences again at
the saved pose instead of storing them.  Correspondences and source
covariances are constants of the function (not differentiated).
"""
from __future__ import annotations

import torch

from . import far


class GicpCost(torch.autograd.Function):
    """cost = GicpCost.apply(src, T, map, cov6, valid, tau, kappa, precision)

    src: [3, n] float32 on the GPU (sensor frame); T: [4, 4] float64 (any
    device), the pose map <- sensor with its rotation block treated as a free
    3 x 3 matrix.  Returns a float64 scalar on T's device.  Gradients: d cost
    / d src ([3, n], float32) and d cost / d T ([4, 4], last row zero)."""

    @staticmethod
    def forward(ctx, src, T, map_, cov6, valid, tau, kappa, precision=far.FAR_PREC_FP32):
        Th = T.detach().to("cpu", torch.float64).numpy()
        lin = far.far_gicp_linearize(map_.h, src.detach(), cov6, valid, Th, tau, kappa,
                                     precision=precision)
        ctx.save_for_backward(src, T)
        ctx.args = (map_, cov6, valid, tau, kappa, precision)
        return torch.tensor(lin["cost"], dtype=torch.float64, device=T.device)

    @staticmethod
    def backward(ctx, g):
        src, T = ctx.saved_tensors
        map_, cov6, valid, tau, kappa, precision = ctx.args
        Th = T.detach().to("cpu", torch.float64).numpy()
        gr = far.far_gicp_gradient(map_.h, src.detach(), cov6, valid, Th, tau, kappa,
                                   precision=precision, want_src=ctx.needs_input_grad[0])
        g_src = g_T = None
        if ctx.needs_input_grad[0]:
            g_src = gr["grad_src"] * g.to(device=src.device, dtype=src.dtype)
        if ctx.needs_input_grad[1]:
            g_T = torch.zeros((4, 4), dtype=torch.float64)
            g_T[:3, :] = torch.from_numpy(gr["grad_T"])
            g_T = g_T.to(T.device) * g.to(device=T.device, dtype=torch.float64)
        return g_src, g_T, None, None, None, None, None, None


def gicp_cost(src, T, map_, cov6, valid, tau, kappa, precision=far.FAR_PREC_FP32):
    return GicpCost.apply(src, T, map_, cov6, valid, tau, kappa, precision)
