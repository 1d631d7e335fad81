"""Plain, slow CPU FP64 oracle for state-to-state GRAPE.

TEST INFRASTRUCTURE. Only tests/, the smoke check and the benchmark's CPU
baseline may import this module; the HIP product path shares no code with it.

The piecewise-constant model of the unitary oracle (GRAPE, Khaneja et al.,
J. Magn. Reson. 172 (2005); hbar = 1), with a state in place of the
propagator (their state-to-state transfer problem):

    psi_0 given (unit vector),  psi_{k+1} = U_k psi_k,   U_k = exp(-i dt H_k)
    chi given (target unit vector)
    g = <chi | psi_N> = chi^dag psi_N,   F = |g|^2
    costates  lam_N = chi,  lam_k = U_k^dag lam_{k+1}
    dg/du[j, k] = lam_{k+1}^dag L(A_k, E_j) psi_k,  A_k = -i dt H_k,  E_j = -i dt H_j
    dF/du[j, k] = 2 Re( conj(g) dg/du[j, k] )

The derivative is the exact one of the piecewise-constant model.  It is the
unitary oracle's <W_k, L(A_k, E_j)>_F with the rank-one W_k = lam_{k+1} psi_k^dag.
Exponentials come from Hermitian eigendecomposition (numpy.linalg.eigh) and
L(A, E) from the Daleckii-Krein formula (Higham, Functions of Matrices, SIAM
2008, Thm. 3.11), in the eigenbasis of H_k:

    lam~ = Q^dag lam_{k+1},  psi~ = Q^dag psi_k,  E~ = Q^dag E_j Q
    dg/du[j, k] = sum_pq conj(lam~_p) Gamma_pq E~_pq psi~_q

with Gamma as in the unitary oracle.  Every step is complex128, with no
blocking or fusion.  Indices: psis[k] is the state before slice k
(psis[0] = psi_0, psis[N] = psi_N); lams[k] is the costate after slice k - 1.
"""
from __future__ import annotations

import numpy as np

from .grape import _dk_gamma, slice_propagators


def forward_states(Us: np.ndarray, psi0: np.ndarray) -> np.ndarray:
    """psis[0] = psi_0 and psis[k + 1] = U_k psis[k]; shape (N + 1, d)."""
    N, d, _ = Us.shape
    psis = np.empty((N + 1, d), dtype=np.complex128)
    psis[0] = np.asarray(psi0, dtype=np.complex128)
    for k in range(N):
        psis[k + 1] = Us[k] @ psis[k]
    return psis


def backward_costates(Us: np.ndarray, chi: np.ndarray) -> np.ndarray:
    """lams[N] = chi and lams[k] = U_k^dag lams[k + 1]; shape (N + 1, d)."""
    N, d, _ = Us.shape
    lams = np.empty((N + 1, d), dtype=np.complex128)
    lams[N] = np.asarray(chi, dtype=np.complex128)
    for k in range(N - 1, -1, -1):
        lams[k] = Us[k].conj().T @ lams[k + 1]
    return lams


def state_overlap(chi: np.ndarray, psiN: np.ndarray):
    """g = <chi | psi_N> and F = |g|^2."""
    g = np.vdot(np.asarray(chi, dtype=np.complex128), psiN)
    return complex(g), float(abs(g) ** 2)


def state_dg(H0, Hc, u, dt, psi0, chi):
    """g = <chi | psi_N>, the complex dg/du[j, k] (m x N) by Daleckii-Krein,
    and psi_N."""
    Hc = np.asarray(Hc, dtype=np.complex128)
    Us, lams_eig, Qs = slice_propagators(H0, Hc, u, dt)
    psis = forward_states(Us, psi0)
    lams = backward_costates(Us, chi)
    g, _ = state_overlap(chi, psis[-1])
    N = Us.shape[0]
    m = Hc.shape[0]
    dg = np.empty((m, N), dtype=np.complex128)
    for k in range(N):
        Q = Qs[k]
        lt = Q.conj().T @ lams[k + 1]
        pt = Q.conj().T @ psis[k]
        gamma = _dk_gamma(lams_eig[k], dt)
        for j in range(m):
            Et = Q.conj().T @ (-1j * dt * Hc[j]) @ Q
            dg[j, k] = lt.conj() @ (gamma * Et) @ pt
    return g, dg, psis[-1]


def state_gradient(H0, Hc, u, dt, psi0, chi):
    """Exact dF/du[j, k] = 2 Re(conj(g) dg/du[j, k]); returns (F, g, grad, psi_N)."""
    g, dg, psiN = state_dg(H0, Hc, u, dt, psi0, chi)
    grad = 2.0 * (np.conj(g) * dg).real
    return float(abs(g) ** 2), g, grad, psiN


def state_ref(problem):
    """Oracle result for a workloads.StateProblem: F, g, grad (m x N), psi_N."""
    F, g, grad, psiN = state_gradient(problem.H0, problem.Hc, problem.u, problem.dt, problem.psi0, problem.chi)
    return {"F": F, "g": g, "grad": grad, "psiN": psiN}
