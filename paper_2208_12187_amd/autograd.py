"""torch.autograd.Function around the libqoc gradient entry point.

The forward pass enqueues the whole GRAPE path (propagators, scans, fidelity
and the adjoint gradient) in one call and keeps the gradient; the backward
pass only scales it by the incoming gradient.  All GPU work runs in libqoc's
kernels; torch provides the tensors and the stream.
"""
from __future__ import annotations

import torch

from . import qoc


class GrapeProblem:
    """Fixed part of a batch of GRAPE problems on one device.

    H0 [B, d, d], Hc [B, m, d, d], V [B, d, d] complex128 tensors; dt a float.
    The runner's workspace is sized for amplitudes of shape [B, m, N].
    ``hbm_budget`` (bytes) turns on checkpointing of stored propagators.
    """

    def __init__(self, H0, Hc, V, dt, N, precision="fp64", hbm_budget=0, chunk=0):
        self.H0 = H0.contiguous()
        self.Hc = Hc.contiguous()
        self.V = V.contiguous()
        self.dt = float(dt)
        self.B, self.d, self.m, self.N = self.H0.shape[0], self.H0.shape[1], self.Hc.shape[1], int(N)
        self.runner = qoc.Runner(self.B, self.d, self.m, self.N, precision, chunk=chunk,
                                 device=self.H0.device, hbm_budget=hbm_budget)

    @staticmethod
    def from_problems(problems, device="cuda", **kw):
        import numpy as np

        H0 = torch.from_numpy(np.stack([p.H0 for p in problems])).to(device)
        Hc = torch.from_numpy(np.stack([p.Hc for p in problems])).to(device)
        V = torch.from_numpy(np.stack([p.V for p in problems])).to(device)
        dts = {p.dt for p in problems}
        Ns = {p.N for p in problems}
        assert len(dts) == 1 and len(Ns) == 1, "a batch shares dt and N"
        return GrapeProblem(H0, Hc, V, dts.pop(), Ns.pop(), **kw)

    def batch(self, u):
        return qoc.Batch(self.H0, self.Hc, u, self.dt, self.V)


class GrapeFidelity(torch.autograd.Function):
    """F = |Tr(V^dag X_N(u))|^2 / d^2 for every problem of the batch."""

    @staticmethod
    def forward(ctx, u, problem: GrapeProblem):
        F, grad = problem.runner.gradient(problem.batch(u.detach().contiguous()))
        ctx.save_for_backward(grad)
        return F

    @staticmethod
    def backward(ctx, gF):
        (grad,) = ctx.saved_tensors
        return gF.to(grad.dtype)[:, None, None] * grad, None


def fidelity(u: torch.Tensor, problem: GrapeProblem) -> torch.Tensor:
    """Differentiable fidelities [B] of amplitudes u [B, m, N] (float64)."""
    return GrapeFidelity.apply(u, problem)
