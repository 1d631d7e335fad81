"""CPU test of the L-BFGS driver, with the oracle's F and gradient standing in
for the GPU path: on a Haar-random target (F starts near 1/d^2, where the
first curvature pairs are rejected and the first quasi-Newton step
overshoots) the driver must keep improving F instead of freezing after a
rejected trial step."""
import numpy as np
import torch

import oracle
from paper_2208_12187_amd import optimize
from workloads import make_config


class _OracleFidelity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, p):
        F, _, grad, _ = oracle.gradient(p.H0, p.Hc, u[0].detach().numpy(), p.dt, p.V)
        ctx.save_for_backward(torch.from_numpy(grad)[None])
        return torch.tensor([F], dtype=torch.float64)

    @staticmethod
    def backward(ctx, dF):
        (grad,) = ctx.saved_tensors
        return dF[:, None, None] * grad, None


def test_lbfgs_keeps_improving_on_a_haar_target(monkeypatch):
    monkeypatch.setattr(optimize, "fidelity", lambda u, p: _OracleFidelity.apply(u, p))
    p = make_config(2, N=60)
    _, hist = optimize.optimise(p, torch.from_numpy(p.u[None]).clone(), iters=25)
    Fs = np.array([h["F"][0] for h in hist])
    assert Fs[0] < 0.01
    assert np.all(np.diff(Fs) >= -1e-12)
    # a driver whose line search cannot backtrack reaches only about 0.0035 here
    assert Fs[-1] > 0.05
    assert Fs[-1] > Fs[-6]
