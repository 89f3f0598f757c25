"""torch.autograd wrapper around a libism handle.

The forward pass is ism_fidelity at the given controls: slice propagators, boundary
rebuild and the objective J[u] = Re<psi(T)|psi_f> - tau/2 sum alpha |u|^2 (Sec. 2); the
boundary states psi(t_n), chi(t_n) stay on the device as the checkpoints.  The backward
pass is ism_gradient: the hand-written adjoint sweeps run slice by slice from those
checkpoints, recomputing the forward states inside each slice, and return
g = (1/tau) dJ/du (Theorem 2 assembles it slice-parallel).  The autograd gradient is
therefore dJ/du = tau g.

The handle must be created with io_device=True (controls and gradients stay on the GPU).
Its stream is ordered against torch's current stream in both directions around every
library call (the controls are ready before the library reads them; J and the gradient are
ready before torch reads them), so forward and backward may run under any torch stream.
"""
from __future__ import annotations

import torch

from ._lib import Problem

__all__ = ["ISMObjective", "ISMControl"]


class ISMObjective(torch.autograd.Function):
    """J = ISMObjective.apply(u, handle): u is a (B, K, C) float64 CUDA tensor; J is (B,)."""

    @staticmethod
    def forward(ctx, u: torch.Tensor, handle: Problem):
        if not handle.io_device:
            raise ValueError("ISMObjective needs a handle created with io_device=True")
        if u.dtype != torch.float64 or not u.is_cuda:
            raise TypeError("controls must be a float64 CUDA tensor")
        uc = u.detach().contiguous()
        cur, hs = torch.cuda.current_stream(), handle.torch_stream
        hs.wait_stream(cur)               # uc is written on cur
        handle.set_controls(uc)
        J, _ = handle.fidelity()
        cur.wait_stream(hs)               # J is written on the handle's stream
        ctx.handle = handle
        ctx.version = handle.version
        ctx.save_for_backward(uc)
        return J.clone()

    @staticmethod
    def backward(ctx, gJ: torch.Tensor):
        (uc,) = ctx.saved_tensors
        h: Problem = ctx.handle
        cur, hs = torch.cuda.current_stream(), h.torch_stream
        hs.wait_stream(cur)
        if h.version != ctx.version:      # the handle was reused: restore this graph's controls
            h.set_controls(uc)
        g = h.gradient()                  # (1/tau) dJ/du, device tensor
        cur.wait_stream(hs)
        tau = h.T / h.K
        return gJ.to(g.dtype)[:, None, None] * g * tau, None


class ISMControl(torch.nn.Module):
    """Controls as an nn.Parameter; forward() returns J per instance.

    Example::

        m = ISMControl(problem_handle, u0)
        opt = torch.optim.Adam(m.parameters(), lr=1e-2)
        for _ in range(n):
            opt.zero_grad(); loss = -m().sum(); loss.backward(); opt.step()
    """

    def __init__(self, handle: Problem, u0):
        super().__init__()
        self.handle = handle
        u = torch.as_tensor(u0, dtype=torch.float64).to("cuda").reshape(handle.B, handle.K,
                                                                           handle.C)
        self.u = torch.nn.Parameter(u.contiguous())

    def forward(self) -> torch.Tensor:
        return ISMObjective.apply(self.u, self.handle)
