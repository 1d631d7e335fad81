"""Control optimisation driver: maximise F with torch.optim.LBFGS (or plain
gradient ascent) through the GrapeFidelity autograd function.

Every objective evaluation is one forward + gradient pass of libqoc.  When
``checkpoint`` is given the driver saves u and the F history to an .npz file
after each iteration and resumes from it (the L-BFGS curvature pairs are
rebuilt after a resume).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from .autograd import GrapeProblem, fidelity


def optimise(problem: GrapeProblem, u0: torch.Tensor, iters: int = 50, method: str = "lbfgs",
             lr: float = 1.0, checkpoint: str | None = None, scale: float | None = None, max_ls: int = 25):
    """Run `iters` optimiser iterations from u0 [B, m, N]; returns (u, history).

    The optimiser works on x = u / scale.  Each amplitude only enters through
    dt * u, so dF/du is O(dt) per entry and an unscaled first L-BFGS step
    (length 1 / |g|_1 in the gradient direction) barely moves u; with the
    default scale = 0.75 sqrt(m N) that first step changes each amplitude by
    about 0.75 / sqrt(m N).

    Each L-BFGS iteration runs a strong-Wolfe line search of at most max_ls
    objective evaluations.

    history: list of dicts {iter, F (list over the batch), evals, seconds};
    entry 0 is the starting point."""
    if scale is None:
        scale = 0.75 * float(np.sqrt(u0.shape[1] * u0.shape[2]))
    x = (u0.detach() / scale).clone().requires_grad_(True)
    history = []
    start_iter = 0
    if checkpoint and os.path.exists(checkpoint):
        z = np.load(checkpoint, allow_pickle=False)
        with torch.no_grad():
            x.copy_(torch.from_numpy(z["u"]).to(x.device) / scale)
        start_iter = int(z["iter"])
        history = json.loads(str(z["history"]))
    evals = [0]

    def objective():
        evals[0] += 1
        return -fidelity(x * scale, problem).sum()

    if method == "lbfgs":
        # One L-BFGS iteration per step() call.  torch gives the line search
        # max_eval minus the evaluations already made in the call, and the
        # default max_eval (5/4 of max_iter) would leave it none: a trial step
        # that does not lower the objective would then be replaced by a zero
        # step, and every later call would retry the same rejected direction.
        opt = torch.optim.LBFGS([x], lr=lr, max_iter=1, max_eval=1 + max_ls, history_size=20,
                                line_search_fn="strong_wolfe")

        def closure():
            opt.zero_grad()
            loss = objective()
            loss.backward()
            return loss
    else:
        opt = torch.optim.SGD([x], lr=lr)
        closure = None

    t0 = time.perf_counter()
    if start_iter == 0 and not history:
        with torch.no_grad():
            F = fidelity(x * scale, problem)
        evals[0] += 1
        history.append({"iter": 0, "F": [float(x) for x in F.cpu()], "evals": evals[0], "seconds": 0.0})
    for it in range(start_iter, iters):
        if closure is not None:
            opt.step(closure)
        else:
            opt.zero_grad()
            loss = objective()
            loss.backward()
            opt.step()
        with torch.no_grad():
            F = fidelity(x * scale, problem)
        evals[0] += 1
        history.append({"iter": it + 1, "F": [float(x) for x in F.cpu()], "evals": evals[0],
                        "seconds": time.perf_counter() - t0})
        if checkpoint:
            np.savez(checkpoint, u=(x.detach() * scale).cpu().numpy(), iter=it + 1, history=json.dumps(history))
    return (x.detach() * scale), history


def main(argv=None):
    ap = argparse.ArgumentParser(description="GRAPE L-BFGS on a spin-chain workload")
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--hbm-budget", type=float, default=0, help="bytes for stored propagators (0: unlimited)")
    ap.add_argument("--method", default="lbfgs", choices=["lbfgs", "ascent"])
    ap.add_argument("--lr", type=float, default=1.0)
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from workloads import make_config

    p = make_config(args.config)
    prob = GrapeProblem.from_problems([p], precision=args.precision, hbm_budget=int(args.hbm_budget))
    u0 = torch.from_numpy(p.u[None]).cuda()
    u, hist = optimise(prob, u0, args.iters, args.method, args.lr)
    print(json.dumps({"config": args.config, "precision": args.precision, "iters": args.iters,
                      "F0": hist[0]["F"][0] if hist else None, "F_final": hist[-1]["F"][0] if hist else None,
                      "evals": hist[-1]["evals"] if hist else 0, "seconds": hist[-1]["seconds"] if hist else 0,
                      "F_trace": [h["F"][0] for h in hist]}))


if __name__ == "__main__":
    main()
