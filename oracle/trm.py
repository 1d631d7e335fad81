"""Plain CPU FP64 oracle for the paper's trust-region method (TRM) and for the
GRAPE least-squares residual it drives.

TEST INFRASTRUCTURE. Only tests/, the smoke check and the benchmark's CPU
baseline may import this module; the HIP product path shares no code with it.

The method (the paper's Sec. 2, Eqs. msqe, mp, lm, pbound, phi, alphaupdate,
accuracy; Alg. 1 overall loop, Alg. 2 Levenberg-Marquardt parameter, Alg. 3
step acceptance and radius update; App. B the SVD solve):

    f(x) = 1/2 r(x)^T r(x),   g = J^T r,   B = J^T J,   scaled J^ = J D^-1
    model  m(w) = f + g^T w + 1/2 w^T B w, trust region |D w| <= Delta
    step   (B^ + alpha I) p = -g^,  alpha (Delta - |p|) = 0,  w = D^-1 p
    SVD    J^ = U S V^T:  p(alpha) = -V (S^2 + alpha)^-1 S U^T r
    phi(alpha) = |p(alpha)| - Delta
    alpha <- alpha - ((phi + Delta) / Delta) (phi / phi')  within [l, u], else
             max(0.001 u, sqrt(l u)); u0 = |g^| / Delta, l0 = -phi(0) / phi'(0)
    gamma = (f(x) - f(x + w)) / (m(0) - m(w)):  > 0.75 accept, Delta <- 2 Delta;
            in [0.25, 0.75] accept, Delta kept; else reject, Delta <- |p| / 4

Readings where the paper is silent or its text garbled (each listed in the
design notes):
  * Alg. 2's loop condition is printed as |phi| <= sigma Delta; the text says
    alpha is updated until |phi| <= sigma Delta, which is what is done here.
  * Alg. 1 and App. B print p = (B^ + alpha I)^-1 g^; Eq. lm fixes the sign,
    p = -(B^ + alpha I)^-1 g^.
  * B^ is singular when J^ has fewer rows than columns or dependent columns
    (always for GRAPE, 2 d^2 residuals and m N + 1 parameters): the alpha = 0
    trial step is then the least-norm one, -B^+ g^ = -V S^-1 U^T r over the
    nonzero singular values, and l0 = 0 (More's rule for a singular B^).
  * D = I, sigma = 0.1, Delta0 = max(|x0|, 1), at most 20 updates of alpha per
    step; the accuracy condition is |g^|_inf <= gtol, a relative decrease of f
    below ftol on an accepted step, or the iteration limit.

GRAPE residual (the least-squares form of the unitary problem): parameters
x = (u[0, 0], ..., u[m-1, N-1], phi), residual
    r(x) = (Re vec(X_N(u) - e^{i phi} V), Im vec(X_N(u) - e^{i phi} V)),
so f = d - Re(e^{-i phi} Tr(V^dag X_N)) and, at the best phi, f = d (1 - sqrt(F)).
Its Jacobian has the columns d vec X_N / d u[j, k] = P_{>k} L(A_k, E_j) X_k,
P_{>k} = U_{N-1} ... U_{k+1}, with L by the Daleckii-Krein formula of the
unitary oracle, and the phi column vec(-i e^{i phi} V).
"""
from __future__ import annotations

import numpy as np

from .grape import backward_products, forward_products, frechet_dk, slice_propagators


# ---------------------------------------------------------------- the method

def svd_step(s: np.ndarray, c: np.ndarray, Vt: np.ndarray, alpha: float) -> np.ndarray:
    """App. B: p(alpha) = -V (S^2 + alpha)^-1 S (U^T r), c = U^T r over the
    kept singular values s, Vt = V^T (rows = right singular vectors)."""
    return -(Vt.T @ (s / (s * s + alpha) * c))


def phi_and_slope(s: np.ndarray, c: np.ndarray, alpha: float, Delta: float):
    """phi(alpha) = |p(alpha)| - Delta and its derivative in alpha."""
    den = s * s + alpha
    pn = np.sqrt(np.sum((s * c / den) ** 2))
    dphi = -np.sum(s * s * c * c / den ** 3) / pn
    return pn - Delta, dphi


def lm_parameter(s, c, Delta, sigma, full_rank, max_iter=20):
    """Alg. 2: alpha > 0 with |phi(alpha)| <= sigma Delta, from alpha_0 = 0."""
    gnorm = np.linalg.norm(s * c)
    upper = gnorm / Delta
    phi0, dphi0 = phi_and_slope(s, c, 0.0, Delta)
    lower = -phi0 / dphi0 if full_rank else 0.0
    alpha = 0.0
    for _ in range(max_iter):
        ph, dph = phi_and_slope(s, c, alpha, Delta)
        if abs(ph) <= sigma * Delta:
            break
        trial = alpha - ((ph + Delta) / Delta) * (ph / dph)
        nxt = trial if lower <= trial <= upper else max(0.001 * upper, np.sqrt(lower * upper))
        lower = max(lower, alpha - ph / dph)
        if ph < 0:
            upper = alpha
        alpha = nxt
    return alpha


def trm(fun, jac, x0, Delta0=None, sigma=0.1, max_iter=50, gtol=1e-10, ftol=1e-12, rank_tol=1e-12,
        callback=None):
    """Alg. 1 with Alg. 2 and Alg. 3 (D = I).  fun(x) -> r, jac(x) -> J.
    Returns (x, info) with info['f'] the accepted f values, info['steps']
    the (gamma, Delta, alpha, accepted) of every iteration."""
    x = np.asarray(x0, dtype=np.float64).copy()
    r = fun(x)
    f = 0.5 * float(r @ r)
    Delta = float(Delta0) if Delta0 is not None else max(float(np.linalg.norm(x)), 1.0)
    info = {"f": [f], "steps": [], "reason": "max_iter"}
    J = jac(x)
    for it in range(max_iter):
        g = J.T @ r
        if np.max(np.abs(g)) <= gtol:
            info["reason"] = "gtol"
            break
        U, s, Vt = np.linalg.svd(J, full_matrices=False)
        keep = s > rank_tol * s[0]
        s, U, Vt = s[keep], U[:, keep], Vt[keep]
        full_rank = bool(keep.all()) and J.shape[0] >= J.shape[1]
        c = U.T @ r
        pt = svd_step(s, c, Vt, 0.0)
        if np.linalg.norm(pt) <= Delta:
            p, alpha = pt, 0.0
        else:
            alpha = lm_parameter(s, c, Delta, sigma, full_rank)
            p = svd_step(s, c, Vt, alpha)
        w = p  # D = I
        Jw = J @ w
        predicted = -(g @ w + 0.5 * Jw @ Jw)  # m(0) - m(w)
        r_new = fun(x + w)
        f_new = 0.5 * float(r_new @ r_new)
        gamma = (f - f_new) / predicted if predicted > 0 else -np.inf
        accepted = gamma >= 0.25
        if gamma > 0.75:
            Delta_new = 2.0 * Delta
        elif gamma >= 0.25:
            Delta_new = Delta
        else:
            Delta_new = 0.25 * float(np.linalg.norm(p))
        info["steps"].append((float(gamma), Delta, float(alpha), bool(accepted)))
        Delta = Delta_new
        if accepted:
            x = x + w
            small = f - f_new <= ftol * f
            r, f = r_new, f_new
            info["f"].append(f)
            if callback:
                callback(it, x, f)
            if small:
                info["reason"] = "ftol"
                break
            J = jac(x)
    return x, info


# ---------------------------------------------------------------- GRAPE residual

def grape_xn_jacobian(H0, Hc, u, dt):
    """X_N and d X_N / d u[j, k] for every (j, k): shape (m, N, d, d)."""
    Hc = np.asarray(Hc, dtype=np.complex128)
    Us, lams, Qs = slice_propagators(H0, Hc, u, dt)
    Xs = forward_products(Us)
    d = Us.shape[1]
    Ps = backward_products(Us, np.eye(d, dtype=np.complex128))  # Ps[k + 1]^dag = U_{N-1} ... U_{k+1}
    m, N = Hc.shape[0], Us.shape[0]
    dX = np.empty((m, N, d, d), dtype=np.complex128)
    for k in range(N):
        left = Ps[k + 1].conj().T
        for j in range(m):
            L = frechet_dk(lams[k], Qs[k], dt, -1j * dt * Hc[j])
            dX[j, k] = left @ L @ Xs[k]
    return Xs[-1], dX


def grape_residual(H0, Hc, u, dt, V, phi):
    """r = (Re vec R, Im vec R) with R = X_N(u) - e^{i phi} V (row-major vec)."""
    Us, _, _ = slice_propagators(H0, Hc, u, dt)
    R = forward_products(Us)[-1] - np.exp(1j * phi) * np.asarray(V)
    return np.concatenate([R.real.ravel(), R.imag.ravel()])


def grape_residual_jacobian(H0, Hc, u, dt, V, phi):
    """J = d r / d (u[0, 0], ..., u[m-1, N-1], phi): shape (2 d^2, m N + 1)."""
    _, dX = grape_xn_jacobian(H0, Hc, u, dt)
    m, N, d, _ = dX.shape
    cols = dX.reshape(m * N, d * d).T
    dphi = (-1j * np.exp(1j * phi) * np.asarray(V)).ravel()[:, None]
    Jc = np.concatenate([cols, dphi], axis=1)
    return np.concatenate([Jc.real, Jc.imag], axis=0)


def grape_trm(problem, phi0=None, **kw):
    """The TRM on the GRAPE residual of a workloads.Problem from its u and
    phi0 (default: the phase of Tr(V^dag X_N(u))).  Returns (u, phi, info)."""
    p = problem
    m, N = p.m, p.N
    if phi0 is None:
        Us, _, _ = slice_propagators(p.H0, p.Hc, p.u, p.dt)
        phi0 = float(np.angle(np.trace(np.asarray(p.V).conj().T @ forward_products(Us)[-1])))
    x0 = np.concatenate([np.asarray(p.u, dtype=np.float64).ravel(), [phi0]])

    def fun(x):
        return grape_residual(p.H0, p.Hc, x[:-1].reshape(m, N), p.dt, p.V, x[-1])

    def jac(x):
        return grape_residual_jacobian(p.H0, p.Hc, x[:-1].reshape(m, N), p.dt, p.V, x[-1])

    x, info = trm(fun, jac, x0, **kw)
    return x[:-1].reshape(m, N), float(x[-1]), info
