"""The paper's trust-region method (Sec. 2, Alg. 1-3, App. B) driving GRAPE.

The least-squares form of the unitary problem: parameters
x = (u[0, 0], ..., u[m-1, N-1], phi) and residual
    r(x) = (Re vec R, Im vec R),   R = X_N(u) - e^{i phi} V,
so f = 1/2 |r|^2 = d - Re(e^{-i phi} Tr(V^dag X_N)), which at the best phase
is d (1 - sqrt(F)).  Minimising f maximises the fidelity.

Where the work runs:
  * X_N: qoc_propagate_dev (libqoc kernels).
  * The Jacobian J (2 d^2 x (m N + 1)): its rows d(X_N)_ab/du come from
    qoc_trace_gradient_dev on a batch of d^2 copies of the problem with the
    targets V_ab = e_a e_b^T (Tr(V_ab^dag X_N) = (X_N)_ab); the phi column is
    vec(-i e^{i phi} V).  J stays in device memory.
  * The thin SVD of J (App. B) is a library call on the device
    (torch.linalg.svd, rocSOLVER), once per accepted step, as the paper does
    it once per update.
  * The scalar work of Alg. 2 and 3 (the LM parameter on the r singular
    values, the gain ratio, the radius) runs on the host, as in the paper.

Readings (where the paper is silent or garbled): Alg. 2 iterates until
|phi(alpha)| <= sigma Delta (its loop condition is printed inverted); the
step is p = -(B^ + alpha I)^-1 g^ (Alg. 1 and App. B drop Eq. lm's sign); a
singular B^ (always here: 2 d^2 residuals, m N + 1 parameters) takes the
least-norm alpha = 0 step and the lower bound l0 = 0; D = I, sigma = 0.1,
Delta0 = max(|x0|, 1); the accuracy condition is |g^|_inf <= gtol, a relative
decrease of f below ftol on an accepted step, or the iteration limit.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import qoc


class GrapeLSQ:
    """Residual and Jacobian of one GRAPE problem on the device."""

    def __init__(self, problem, precision="fp64", device="cuda"):
        import torch

        p = problem
        self.d, self.m, self.N, self.dt = p.d, p.m, p.N, p.dt
        self.precision = precision
        self.device = device
        c128 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(device)
        self.H0, self.Hc, self.V = c128(p.H0), c128(p.Hc), c128(p.V)
        d, n2 = self.d, self.d * self.d
        # batch of d^2 copies with the unit targets e_a e_b^T, row-major (a, b)
        self.Hb = self.H0.unsqueeze(0).expand(n2, d, d).contiguous()
        self.Hcb = self.Hc.unsqueeze(0).expand(n2, self.m, d, d).contiguous()
        E = torch.zeros((n2, d, d), dtype=torch.complex128, device=device)
        idx = torch.arange(n2, device=device)
        E[idx, idx // d, idx % d] = 1.0
        self.E = E
        self.one = qoc.Runner(1, d, self.m, self.N, precision, device=device)
        self.many = qoc.Runner(n2, d, self.m, self.N, precision, device=device)
        self.evals = 0
        self.jacobians = 0

    def _u(self, x):
        return x[:-1].reshape(1, self.m, self.N)

    def residual(self, x):
        """r(x) as a float64 device vector of length 2 d^2."""
        import torch

        b = qoc.Batch(self.H0[None], self.Hc[None], self._u(x), self.dt, None)
        XN = self.one.propagate(b)[0]
        R = XN - torch.exp(1j * x[-1]) * self.V
        self.evals += 1
        return torch.cat([R.real.reshape(-1), R.imag.reshape(-1)])

    def jacobian(self, x):
        """J(x) on the device, shape (2 d^2, m N + 1)."""
        import torch

        n2 = self.d * self.d
        ub = self._u(x).expand(n2, self.m, self.N).contiguous()
        b = qoc.Batch(self.Hb, self.Hcb, ub, self.dt, self.E)
        _, dg = self.many.trace_gradient(b)                      # (d^2, m, N): d(X_N)_ab / du
        rows = dg.reshape(n2, self.m * self.N)
        dphi = (-1j * torch.exp(1j * x[-1]) * self.V).reshape(n2, 1)
        Jc = torch.cat([rows, dphi], dim=1)
        self.jacobians += 1
        return torch.cat([Jc.real, Jc.imag], dim=0)

    def trace_gradient(self, x, W):
        """d Tr(W^dag X_N) / du for one d x d device matrix W (complex m x N)."""
        b = qoc.Batch(self.H0[None], self.Hc[None], self._u(x), self.dt, W[None].contiguous())
        _, dg = self.one.trace_gradient(b)
        return dg[0]


def _phi_slope(s, c, alpha, Delta):
    """|p(alpha)| - Delta and its alpha-derivative for p = -V (S^2+alpha)^-1 S c."""
    q = s * s + alpha
    w = s * c / q
    norm = math.sqrt(float(np.dot(w, w)))
    slope = -float(np.sum((s * c) ** 2 / q ** 3)) / norm
    return norm - Delta, slope


def lm_alpha(s, c, Delta, sigma, nonsingular, max_iter=20):
    """Alg. 2 on the host: the LM parameter that puts |p| within sigma Delta
    of Delta, starting from alpha = 0 with More's safeguards."""
    hi = math.sqrt(float(np.sum((s * c) ** 2))) / Delta
    ph0, sl0 = _phi_slope(s, c, 0.0, Delta)
    lo = -ph0 / sl0 if nonsingular else 0.0
    alpha = 0.0
    for _ in range(max_iter):
        ph, sl = _phi_slope(s, c, alpha, Delta)
        if abs(ph) <= sigma * Delta:
            break
        cand = alpha - (ph + Delta) / Delta * ph / sl
        nxt = cand if lo <= cand <= hi else max(1e-3 * hi, math.sqrt(lo * hi))
        lo = max(lo, alpha - ph / sl)
        hi = alpha if ph < 0 else hi
        alpha = nxt
    return alpha


def trm_grape(problem, precision="fp64", max_iter=30, gtol=1e-10, ftol=1e-12, sigma=0.1, Delta0=None,
              phi0=None, rank_rtol=1e-12, device="cuda", log=None):
    """Fit the controls of a workloads.Problem by the trust-region method.
    Returns (u, phi, info): info holds f per accepted step, the fidelity
    F = |Tr(V^dag X_N)|^2 / d^2 per accepted step, the per-iteration
    (gamma, Delta, alpha, accepted), Jacobian and residual counts, times."""
    import torch

    t0 = time.perf_counter()
    lsq = GrapeLSQ(problem, precision, device)
    d = lsq.d
    u0 = torch.from_numpy(np.ascontiguousarray(problem.u, dtype=np.float64)).to(device).reshape(-1)
    if phi0 is None:
        b = qoc.Batch(lsq.H0[None], lsq.Hc[None], u0.reshape(1, lsq.m, lsq.N), lsq.dt, None)
        XN = lsq.one.propagate(b)[0]
        phi0 = float(torch.angle(torch.sum(lsq.V.conj() * XN)))
    x = torch.cat([u0, torch.tensor([phi0], dtype=torch.float64, device=device)])
    r = lsq.residual(x)
    f = 0.5 * float(r @ r)
    Delta = float(Delta0) if Delta0 is not None else max(float(torch.linalg.norm(x)), 1.0)

    def F_of(x):
        b = qoc.Batch(lsq.H0[None], lsq.Hc[None], x[:-1].reshape(1, lsq.m, lsq.N), lsq.dt, None)
        XN = lsq.one.propagate(b)[0]
        g = torch.sum(lsq.V.conj() * XN)
        return float(abs(g) ** 2) / d ** 2

    info = {"f": [f], "F": [F_of(x)], "steps": [], "reason": "max_iter", "svd_s": 0.0, "jac_s": 0.0}
    tj = time.perf_counter()
    J = lsq.jacobian(x)
    torch.cuda.synchronize()
    info["jac_s"] += time.perf_counter() - tj
    svd = None  # the SVD of the current J; a rejected step keeps x, J and it
    for it in range(max_iter):
        g = J.T @ r
        if float(g.abs().max()) <= gtol:
            info["reason"] = "gtol"
            break
        if svd is None:
            ts = time.perf_counter()
            U, s, Vh = torch.linalg.svd(J, full_matrices=False)
            torch.cuda.synchronize()
            info["svd_s"] += time.perf_counter() - ts
            keep = s > rank_rtol * s[0]
            svd = (U[:, keep], s[keep], Vh[keep], bool(keep.all()) and J.shape[0] >= J.shape[1])
        U, s, Vh, nonsingular = svd
        c = (U.T @ r)
        s_h, c_h = s.cpu().numpy(), c.cpu().numpy()
        p = -(Vh.T @ (s / (s * s) * c))
        if float(torch.linalg.norm(p)) <= Delta:
            alpha = 0.0
        else:
            alpha = lm_alpha(s_h, c_h, Delta, sigma, nonsingular)
            p = -(Vh.T @ (s / (s * s + alpha) * c))
        Jp = J @ p
        predicted = -float(g @ p + 0.5 * (Jp @ Jp))
        r_new = lsq.residual(x + p)
        f_new = 0.5 * float(r_new @ r_new)
        gain = (f - f_new) / predicted if predicted > 0 else -math.inf
        accepted = gain >= 0.25
        pn = float(torch.linalg.norm(p))
        info["steps"].append((float(gain), Delta, float(alpha), bool(accepted)))
        Delta = 2.0 * Delta if gain > 0.75 else (Delta if gain >= 0.25 else 0.25 * pn)
        if accepted:
            x = x + p
            small = f - f_new <= ftol * f
            r, f = r_new, f_new
            info["f"].append(f)
            info["F"].append(F_of(x))
            if log:
                log(f"[trm] iter {it}: f = {f:.6e}, F = {info['F'][-1]:.8f}, Delta = {Delta:.3e}, alpha = {alpha:.3e}")
            if small:
                info["reason"] = "ftol"
                break
            tj = time.perf_counter()
            J = lsq.jacobian(x)
            svd = None
            torch.cuda.synchronize()
            info["jac_s"] += time.perf_counter() - tj
    info["jacobians"] = lsq.jacobians
    info["residuals"] = lsq.evals
    info["seconds"] = time.perf_counter() - t0
    xh = x.cpu().numpy()
    return xh[:-1].reshape(lsq.m, lsq.N), float(xh[-1]), info
