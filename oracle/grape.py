"""Plain, slow CPU FP64 oracle for piecewise-constant GRAPE.

TEST INFRASTRUCTURE. Only tests/, the smoke check and the benchmark's CPU
baseline may import this module; the HIP product path shares no code with it.

What it computes (GRAPE, Khaneja et al., J. Magn. Reson. 172 (2005), with
hbar = 1 and the exact derivative of the piecewise-constant model):

    H_k   = H0 + sum_j u[j, k] H_j                       (slice Hamiltonian)
    U_k   = exp(-i dt H_k)                                (slice propagator)
    X_0   = I,  X_{k+1} = U_k X_k        (slice 0 acts first, X_N = U_{N-1}...U_0)
    B_N   = V,  B_k     = U_k^dag B_{k+1}
    g     = Tr(V^dag X_N),   F = |g|^2 / d^2               (phase-insensitive fidelity)
    dF/du[j, k] = (2 / d^2) Re( conj(g) * dg/du[j, k] )
    dg/du[j, k] = Tr( B_{k+1}^dag  L(A_k, E_j)  X_k ),  A_k = -i dt H_k,  E_j = -i dt H_j

L(A, E) is the Frechet derivative of the matrix exponential at A in the
direction E.  The oracle evaluates exponentials by Hermitian
eigendecomposition (LAPACK zheevd through numpy.linalg.eigh) and the
Frechet derivative by the Daleckii-Krein divided-difference formula
(Higham, Functions of Matrices, SIAM 2008, Thm. 3.11):

    A = Q diag(a) Q^dag,  L(A, E) = Q (Gamma o (Q^dag E Q)) Q^dag,
    Gamma_pq = (e^{a_p} - e^{a_q}) / (a_p - a_q)   (= e^{a_p} when a_p = a_q).

For a_p = -i dt lambda_p this equals
    exp(-i dt (lambda_p + lambda_q) / 2) * sinc(dt (lambda_p - lambda_q) / 2),
sinc(x) = sin(x)/x, which stays accurate for the degenerate spectra of spin
chains.  Every step is done in complex128 with no blocking or fusion.

Indices are 0-based in code: slice k acts after slices 0..k-1; Xs[k] is the
product of the slices before k and Bs[k + 1] the backward product after it.
"""
from __future__ import annotations

import numpy as np


def slice_hamiltonians(H0: np.ndarray, Hc: np.ndarray, u: np.ndarray) -> np.ndarray:
    """H_k = H0 + sum_j u[j, k] H_j for every slice k; shape (N, d, d)."""
    H0 = np.asarray(H0, dtype=np.complex128)
    Hc = np.asarray(Hc, dtype=np.complex128)
    u = np.asarray(u, dtype=np.float64)
    return H0[None, :, :] + np.einsum("jk,jab->kab", u, Hc)


def expm_herm(H: np.ndarray, dt: float):
    """exp(-i dt H) for Hermitian H by eigendecomposition.

    Returns (U, lam, Q) with H = Q diag(lam) Q^dag and
    U = Q diag(exp(-i dt lam)) Q^dag."""
    lam, Q = np.linalg.eigh(H)
    U = (Q * np.exp(-1j * dt * lam)[None, :]) @ Q.conj().T
    return U, lam, Q


def slice_propagators(H0, Hc, u, dt):
    """U_k = exp(-i dt H_k) for all slices; also the eigenpairs of every H_k."""
    Hs = slice_hamiltonians(H0, Hc, u)
    Us, lams, Qs = [], [], []
    for Hk in Hs:
        U, lam, Q = expm_herm(Hk, dt)
        Us.append(U)
        lams.append(lam)
        Qs.append(Q)
    return np.array(Us), np.array(lams), np.array(Qs)


def forward_products(Us: np.ndarray) -> np.ndarray:
    """Xs[0] = I and Xs[k + 1] = U_k Xs[k]; shape (N + 1, d, d)."""
    N, d, _ = Us.shape
    Xs = np.empty((N + 1, d, d), dtype=np.complex128)
    Xs[0] = np.eye(d, dtype=np.complex128)
    for k in range(N):
        Xs[k + 1] = Us[k] @ Xs[k]
    return Xs


def backward_products(Us: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Bs[N] = V and Bs[k] = U_k^dag Bs[k + 1]; shape (N + 1, d, d)."""
    N, d, _ = Us.shape
    Bs = np.empty((N + 1, d, d), dtype=np.complex128)
    Bs[N] = np.asarray(V, dtype=np.complex128)
    for k in range(N - 1, -1, -1):
        Bs[k] = Us[k].conj().T @ Bs[k + 1]
    return Bs


def fidelity(V: np.ndarray, XN: np.ndarray):
    """g = Tr(V^dag X_N) and F = |g|^2 / d^2."""
    d = V.shape[0]
    g = np.trace(np.asarray(V).conj().T @ XN)
    return complex(g), float(abs(g) ** 2 / d ** 2)


def frechet_dk(lam: np.ndarray, Q: np.ndarray, dt: float, E: np.ndarray) -> np.ndarray:
    """L(A, E) for A = -i dt H, H = Q diag(lam) Q^dag (Daleckii-Krein)."""
    gamma = _dk_gamma(lam, dt)
    Et = Q.conj().T @ E @ Q
    return Q @ (gamma * Et) @ Q.conj().T


def _dk_gamma(lam: np.ndarray, dt: float) -> np.ndarray:
    """Gamma_pq = exp(-i dt (l_p + l_q)/2) sinc(dt (l_p - l_q)/2)."""
    lp = lam[:, None]
    lq = lam[None, :]
    x = dt * (lp - lq) / 2.0
    # numpy.sinc(t) = sin(pi t)/(pi t), so sin(x)/x = numpy.sinc(x / pi).
    return np.exp(-1j * dt * (lp + lq) / 2.0) * np.sinc(x / np.pi)


def gradient(H0, Hc, u, dt, V):
    """Exact dF/du[j, k] by Daleckii-Krein; returns (F, g, grad, X_N).

    dg/du[j, k] = <W_k, L(A_k, E_j)>_F with W_k = B_{k+1} X_k^dag and
    <X, Y>_F = Tr(X^dag Y); in the eigenbasis of H_k this is
    sum_pq conj((Q^dag W_k Q)_pq) Gamma_pq (Q^dag E_j Q)_pq."""
    Hc = np.asarray(Hc, dtype=np.complex128)
    V = np.asarray(V, dtype=np.complex128)
    Us, lams, Qs = slice_propagators(H0, Hc, u, dt)
    Xs = forward_products(Us)
    Bs = backward_products(Us, V)
    g, F = fidelity(V, Xs[-1])
    N = Us.shape[0]
    m, d = Hc.shape[0], Hc.shape[1]
    grad = np.empty((m, N), dtype=np.float64)
    for k in range(N):
        Q = Qs[k]
        W = Bs[k + 1] @ Xs[k].conj().T
        Wt = Q.conj().T @ W @ Q
        gamma = _dk_gamma(lams[k], dt)
        for j in range(m):
            Et = Q.conj().T @ (-1j * dt * Hc[j]) @ Q
            dg = np.sum(Wt.conj() * gamma * Et)
            grad[j, k] = 2.0 / d ** 2 * (np.conj(g) * dg).real
    return F, g, grad, Xs[-1]


def grape_ref(problem):
    """Oracle result for a workloads.Problem: F, g, grad (m x N), X_N."""
    F, g, grad, XN = gradient(problem.H0, problem.Hc, problem.u, problem.dt, problem.V)
    return {"F": F, "g": g, "grad": grad, "XN": XN}


def fidelity_ref(problem):
    """Oracle F, g and X_N without the gradient."""
    Us, _, _ = slice_propagators(problem.H0, problem.Hc, problem.u, problem.dt)
    XN = forward_products(Us)[-1]
    g, F = fidelity(problem.V, XN)
    return {"F": F, "g": g, "XN": XN}
